// Host side of the hyperparameter optimisation (paper, Sec. "Parallel
// Optimization" and Sec. "Parallel Line Search"): BFGS on f(theta) with the
// exact adjoint gradient, and in every iteration a parallel line search -- the
// candidate points of the search interval and two stabilising points on the
// other side of theta_l evaluated in one batched call, a quadratic fitted to
// their values by robust regression with bisquare weights, and its minimiser
// on the interval taken as the next iterate.
//
// Only the evaluations touch the GPU (through the library's own C ABI); the
// fit and the quasi-Newton update are a few dozen host flops.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/inla_bta.h"
#include "inla_internal.h"

using inla::set_last_error;

namespace {

constexpr int kDim = 4;
// Tukey's bisquare tuning constant (95% efficiency at the normal model) and
// the MAD-to-standard-deviation factor of the normal distribution.
constexpr double kBisquareC = 4.685;
constexpr double kMadNormal = 0.6744897501960817;

double median(std::vector<double> v) {
  if (v.empty()) return 0.0;
  const size_t h = v.size() / 2;
  std::nth_element(v.begin(), v.begin() + h, v.end());
  const double hi = v[h];
  if (v.size() % 2) return hi;
  return 0.5 * (hi + *std::max_element(v.begin(), v.begin() + h));
}

// Weighted least squares for q(u) = c0 + c1 u + c2 u^2 on the scaled abscissa
// u = (x - xm) / xs: the 3 x 3 normal equations solved by Cholesky.  Returns
// false when fewer than three points carry weight or the system is singular.
bool wls_quadratic(const std::vector<double> &u, const std::vector<double> &y,
                   const std::vector<double> &w, double c[3]) {
  double A[3][3] = {}, r[3] = {};
  int used = 0;
  for (size_t i = 0; i < u.size(); ++i) {
    if (!(w[i] > 0.0)) continue;
    ++used;
    const double p[3] = {1.0, u[i], u[i] * u[i]};
    for (int a = 0; a < 3; ++a) {
      r[a] += w[i] * p[a] * y[i];
      for (int b = 0; b < 3; ++b) A[a][b] += w[i] * p[a] * p[b];
    }
  }
  if (used < 3) return false;
  double L[3][3] = {};
  for (int j = 0; j < 3; ++j) {
    double d = A[j][j];
    for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
    if (!(d > 1e-14 * A[j][j]) || !(d > 0.0)) return false;
    L[j][j] = std::sqrt(d);
    for (int i = j + 1; i < 3; ++i) {
      double v = A[i][j];
      for (int k = 0; k < j; ++k) v -= L[i][k] * L[j][k];
      L[i][j] = v / L[j][j];
    }
  }
  double z[3];
  for (int i = 0; i < 3; ++i) {
    double v = r[i];
    for (int k = 0; k < i; ++k) v -= L[i][k] * z[k];
    z[i] = v / L[i][i];
  }
  for (int i = 2; i >= 0; --i) {
    double v = z[i];
    for (int k = i + 1; k < 3; ++k) v -= L[k][i] * c[k];
    c[i] = v / L[i][i];
  }
  return true;
}

}  // namespace

extern "C" {

inla_status inla_robust_quadratic_fit(const double *x, const double *y, int32_t n, double *coef,
                                      double *weights_or_null) {
  set_last_error(INLA_OK, "");
  if (!x || !y || !coef || n < 3) return set_last_error(INLA_ERR_ARG, "need x, y, coef and n >= 3");
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(x[i]) || !std::isfinite(y[i]))
      return set_last_error(INLA_ERR_ARG, "non-finite point");
  // scaled abscissa for a well-conditioned system
  double xm = 0.0;
  for (int i = 0; i < n; ++i) xm += x[i];
  xm /= n;
  double xs = 0.0;
  for (int i = 0; i < n; ++i) xs = std::max(xs, std::fabs(x[i] - xm));
  if (!(xs > 0.0)) return set_last_error(INLA_ERR_ARG, "all abscissae are equal");
  std::vector<double> u(n), yy(y, y + n), w(n, 1.0), r(n), absr(n);
  for (int i = 0; i < n; ++i) u[i] = (x[i] - xm) / xs;
  double c[3] = {0.0, 0.0, 0.0};
  if (!wls_quadratic(u, yy, w, c)) return set_last_error(INLA_ERR_ARG, "fewer than three distinct points");
  double ymax = 0.0;
  for (int i = 0; i < n; ++i) ymax = std::max(ymax, std::fabs(y[i]));
  // iteratively reweighted least squares with bisquare weights
  for (int it = 0; it < 200; ++it) {
    for (int i = 0; i < n; ++i) {
      r[i] = yy[i] - (c[0] + c[1] * u[i] + c[2] * u[i] * u[i]);
      absr[i] = std::fabs(r[i]);
    }
    const double s = median(absr) / kMadNormal;
    std::vector<double> wn(n);
    if (!(s > 1e-15 * std::max(ymax, 1e-300))) {
      // (the limit of the bisquare weights as the scale goes to zero: points
      // on the fit keep weight one, every other point drops out)
      const double tol = 1e-13 * std::max(ymax, 1e-300);
      for (int i = 0; i < n; ++i) wn[i] = absr[i] <= tol ? 1.0 : 0.0;
    } else {
      for (int i = 0; i < n; ++i) {
        const double q = r[i] / (kBisquareC * s);
        wn[i] = std::fabs(q) < 1.0 ? (1.0 - q * q) * (1.0 - q * q) : 0.0;
      }
    }
    double dw = 0.0;
    for (int i = 0; i < n; ++i) dw = std::max(dw, std::fabs(wn[i] - w[i]));
    w.swap(wn);
    double cn[3];
    if (!wls_quadratic(u, yy, w, cn)) break;   // keep the last fit
    std::memcpy(c, cn, sizeof(c));
    if (dw < 1e-12) break;
  }
  // back to the unscaled abscissa: q(x) = c0 + c1 (x-xm)/xs + c2 ((x-xm)/xs)^2
  const double a2 = c[2] / (xs * xs);
  const double a1 = c[1] / xs - 2.0 * a2 * xm;
  const double a0 = c[0] - c[1] * xm / xs + a2 * xm * xm;
  coef[0] = a0;
  coef[1] = a1;
  coef[2] = a2;
  if (weights_or_null)
    for (int i = 0; i < n; ++i) weights_or_null[i] = w[i];
  return INLA_OK;
}

inla_status inla_bfgs_minimize(const inla_model *model, const double *theta0, const inla_bfgs_opts *opts,
                               inla_bfgs_result *res, double *history_or_null, void *hip_stream) {
  set_last_error(INLA_OK, "");
  if (!model || !theta0 || !res) return set_last_error(INLA_ERR_ARG, "need model, theta0 and res");
  for (int k = 0; k < kDim; ++k)
    if (!std::isfinite(theta0[k])) return set_last_error(INLA_ERR_ARG, "theta0 is not finite");
  const int max_iter = (opts && opts->max_iter > 0) ? opts->max_iter : 300;
  const int npts = (opts && opts->n_points > 0) ? opts->n_points : 6;
  const double gamma0 = (opts && opts->gamma > 0.0) ? opts->gamma : 1.0;
  const double gtol = (opts && opts->gtol > 0.0) ? opts->gtol : 1e-6;
  const double ftol = (opts && opts->ftol > 0.0) ? opts->ftol : 1e-13;
  const inla_opts *eo = opts ? opts->eval_opts : nullptr;
  const double max_step = (opts && opts->max_step > 0.0) ? opts->max_step : 2.0;
  if (npts > 62) return set_last_error(INLA_ERR_ARG, "n_points above 62");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  std::memset(res, 0, sizeof(*res));

  // device buffers: the candidate batch and its outputs
  const int cap = npts + 2;
  double *d_th = nullptr, *d_f = nullptr, *d_g = nullptr;
  int *d_st = nullptr;
  if (hipMalloc(&d_th, (size_t)cap * kDim * 8) != hipSuccess || hipMalloc(&d_f, (size_t)cap * 8) != hipSuccess ||
      hipMalloc(&d_g, (size_t)kDim * 8) != hipSuccess || hipMalloc(&d_st, (size_t)cap * 4) != hipSuccess) {
    (void)hipGetLastError();
    if (d_th) (void)hipFree(d_th);
    if (d_f) (void)hipFree(d_f);
    if (d_g) (void)hipFree(d_g);
    if (d_st) (void)hipFree(d_st);
    return set_last_error(INLA_ERR_NOMEM, "optimizer buffers");
  }
  std::vector<const inla_model *> ms(cap, model);
  inla_status rc = INLA_OK;

  // f and grad f at one point (host in, host out)
  auto eval_grad = [&](const double *th, double &f, double *g, int &st) -> inla_status {
    if (hipMemcpyAsync(d_th, th, kDim * 8, hipMemcpyHostToDevice, s) != hipSuccess)
      return set_last_error(INLA_ERR_HIP, "optimizer copy to the device");
    const inla_status e = inla_eval_f_grad(ms.data(), 1, d_th, d_f, d_g, nullptr, nullptr, d_st, eo, s);
    if (e != INLA_OK) return e;
    if (hipMemcpyAsync(&f, d_f, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(g, d_g, kDim * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&st, d_st, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return set_last_error(INLA_ERR_HIP, "optimizer copy to the host");
    ++res->grad_evals;
    return INLA_OK;
  };
  // f at a batch of points in one call
  auto eval_batch = [&](const std::vector<double> &th, std::vector<double> &f, std::vector<int> &st)
      -> inla_status {
    const int k = (int)(th.size() / kDim);
    if (hipMemcpyAsync(d_th, th.data(), th.size() * 8, hipMemcpyHostToDevice, s) != hipSuccess)
      return set_last_error(INLA_ERR_HIP, "optimizer copy to the host");
    const inla_status e = inla_eval_f(ms.data(), k, d_th, d_f, nullptr, nullptr, d_st, eo, s);
    if (e != INLA_OK) return e;
    f.resize(k);
    st.resize(k);
    if (hipMemcpyAsync(f.data(), d_f, (size_t)k * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(st.data(), d_st, (size_t)k * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return set_last_error(INLA_ERR_HIP, "optimizer copy to the host");
    res->f_evals += k;
    return INLA_OK;
  };
  auto gnorm = [](const double *g) {
    double m = 0.0;
    for (int k = 0; k < kDim; ++k) m = std::max(m, std::fabs(g[k]));
    return m;
  };

  double th[kDim], g[kDim], f = 0.0;
  int st = 0;
  std::memcpy(th, theta0, sizeof(th));
  rc = eval_grad(th, f, g, st);
  if (rc == INLA_OK && (st != 0 || !std::isfinite(f)))
    rc = set_last_error(INLA_ERR_NOT_SPD, "f cannot be evaluated at theta0");
  // inverse Hessian approximation H (B^{-1}); the first direction has unit length
  double H[kDim][kDim] = {};
  const double g0 = gnorm(g);
  for (int k = 0; k < kDim; ++k) H[k][k] = g0 > 0.0 ? 1.0 / g0 : 1.0;
  bool first_update = true;
  double gamma = gamma0;
  int reason = 2;   // max iterations unless something else stops it
  int it = 0;
  auto record = [&](double alpha) {
    if (!history_or_null) return;
    double *h = history_or_null + (size_t)it * 8;
    h[0] = f;
    h[1] = gnorm(g);
    h[2] = alpha;
    for (int k = 0; k < kDim; ++k) h[3 + k] = th[k];
    h[7] = res->f_evals;
  };
  if (rc == INLA_OK) record(0.0);
  // the step to (tn, gn, ff): BFGS update of the inverse Hessian with
  // s = theta+ - theta, y = grad+ - grad (skipped unless s^T y > 0), then the
  // new iterate
  double last_alpha = 0.0;
  auto accept = [&](const double *tn, const double *gn, double ff, double alpha) {
    last_alpha = alpha;
    double sv[kDim], yv[kDim], sy = 0.0, yy = 0.0;
    for (int k = 0; k < kDim; ++k) {
      sv[k] = tn[k] - th[k];
      yv[k] = gn[k] - g[k];
      sy += sv[k] * yv[k];
      yy += yv[k] * yv[k];
    }
    if (sy > 0.0 && yy > 0.0) {
      if (first_update) {
        // the scaling of the initial matrix by s^T y / y^T y
        for (int a = 0; a < kDim; ++a)
          for (int b = 0; b < kDim; ++b) H[a][b] = a == b ? sy / yy : 0.0;
        first_update = false;
      }
      const double rho = 1.0 / sy;
      double Hy[kDim], yHy = 0.0;
      for (int a = 0; a < kDim; ++a) {
        Hy[a] = 0.0;
        for (int b = 0; b < kDim; ++b) Hy[a] += H[a][b] * yv[b];
        yHy += yv[a] * Hy[a];
      }
      for (int a = 0; a < kDim; ++a)
        for (int b = 0; b < kDim; ++b)
          H[a][b] += -rho * (Hy[a] * sv[b] + sv[a] * Hy[b]) + (rho * rho * yHy + rho) * sv[a] * sv[b];
    }
    const double df = f - ff;
    std::memcpy(th, tn, sizeof(th));
    std::memcpy(g, gn, sizeof(g));
    f = ff;
    ++it;
    record(alpha);
    if (df <= ftol * std::max(1.0, std::fabs(f))) reason = 1;
  };
  while (rc == INLA_OK && it < max_iter) {
    if (gnorm(g) <= gtol) {
      reason = 0;
      break;
    }
    // search direction p = H grad f; the interval I = (theta, theta - gamma p)
    double p[kDim];
    for (int a = 0; a < kDim; ++a) {
      p[a] = 0.0;
      for (int b = 0; b < kDim; ++b) p[a] += H[a][b] * g[b];
    }
    double slope = 0.0;   // d f(theta - alpha p) / d alpha at 0
    for (int k = 0; k < kDim; ++k) slope -= g[k] * p[k];
    if (!(slope < 0.0)) {
      // not a descent direction (H lost positive definiteness): restart
      for (int a = 0; a < kDim; ++a)
        for (int b = 0; b < kDim; ++b) H[a][b] = a == b ? 1.0 / std::max(gnorm(g), 1e-300) : 0.0;
      continue;
    }
    // the interval of this iteration: gamma, shortened so that no hyperparameter
    // moves by more than max_step
    double pmax = 0.0;
    for (int k = 0; k < kDim; ++k) pmax = std::max(pmax, std::fabs(p[k]));
    double gam = gamma;
    if (gam * pmax > max_step) gam = max_step / pmax;
    // candidate step lengths: npts on the interval, two stabilising ones on
    // the other side of theta, close to it
    bool moved = false;
    for (int attempt = 0; attempt < 8 && !moved && rc == INLA_OK; ++attempt) {
      std::vector<double> alphas{-gam / 4.0, -gam / 8.0};
      for (int i = 1; i <= npts; ++i) alphas.push_back(gam * i / npts);
      std::vector<double> pts;
      for (double al : alphas)
        for (int k = 0; k < kDim; ++k) pts.push_back(th[k] - al * p[k]);
      std::vector<double> fv;
      std::vector<int> sv;
      rc = eval_batch(pts, fv, sv);
      if (rc != INLA_OK) break;
      // points for the fit: theta itself and every candidate with a value
      std::vector<double> xa{0.0}, ya{f};
      double best_alpha = 0.0, best_f = f;
      for (size_t i = 0; i < alphas.size(); ++i)
        if (sv[i] == 0 && std::isfinite(fv[i])) {
          xa.push_back(alphas[i]);
          ya.push_back(fv[i]);
          if (alphas[i] > 0.0 && fv[i] < best_f) {
            best_f = fv[i];
            best_alpha = alphas[i];
          }
        }
      // the minimiser of the robust quadratic on the interval (0, gam]
      double alpha_q = 0.0;
      double c[3];
      if (xa.size() >= 4 &&
          inla_robust_quadratic_fit(xa.data(), ya.data(), (int)xa.size(), c, nullptr) == INLA_OK) {
        if (c[2] > 0.0) alpha_q = std::min(std::max(-c[1] / (2.0 * c[2]), 0.0), gam);
        else alpha_q = (c[1] * gam + c[2] * gam * gam < 0.0) ? gam : 0.0;
      }
      // the fit's minimiser, unless an evaluated candidate is lower; then that one
      std::vector<double> tries;
      if (alpha_q > 0.0) tries.push_back(alpha_q);
      if (best_alpha > 0.0 && best_alpha != alpha_q) tries.push_back(best_alpha);
      for (size_t ti = 0; ti < tries.size() && !moved; ++ti) {
        const double alpha = tries[ti];
        double tn[kDim], gn[kDim], ff = 0.0;
        int sn = 0;
        for (int k = 0; k < kDim; ++k) tn[k] = th[k] - alpha * p[k];
        rc = eval_grad(tn, ff, gn, sn);
        if (rc != INLA_OK) break;
        const bool lower = sn == 0 && std::isfinite(ff) && ff < f;
        if (!lower || (ti == 0 && alpha == alpha_q && best_alpha > 0.0 && best_f < ff)) continue;
        accept(tn, gn, ff, alpha);
        moved = true;
      }
      // nothing on the interval decreased f: a shorter interval
      if (!moved) gam *= 0.25;
    }
    if (rc != INLA_OK) break;
    if (!moved) {
      reason = gnorm(g) <= gtol ? 0 : 3;
      break;
    }
    if (reason == 1) break;
    // the next interval reaches twice the step just taken (at least gamma0):
    // a step at the end of the interval asks for a longer one
    gamma = std::max(gamma0, 2.0 * last_alpha);
  }
  if (rc == INLA_OK && reason == 2 && gnorm(g) <= gtol) reason = 0;
  (void)hipStreamSynchronize(s);
  (void)hipFree(d_th);
  (void)hipFree(d_f);
  (void)hipFree(d_g);
  (void)hipFree(d_st);
  std::memcpy(res->theta, th, sizeof(th));
  std::memcpy(res->grad, g, sizeof(g));
  res->f = f;
  res->iterations = it;
  res->reason = reason;
  return rc;
}

}  // extern "C"
