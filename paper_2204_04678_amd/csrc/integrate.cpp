// Host side of the integration step after the mode search (paper, Sec.
// "Latent Gaussian Models", Sec. "Approximating pi(x_i | y)" with eq.
// LatParam, Sec. "Parallelization of Function Evaluations"): the Hessian at
// the mode from differences of the adjoint gradient, the standardised grid
// of points around the mode, the quadrature over theta, and the latent
// marginals as the weighted mixture of the Gaussian conditionals at the
// points.  Every evaluation is a batched call of the library's own C ABI;
// only the choices of points and the 4-dimensional arithmetic are on the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <vector>

#include "../../include/inla_bta.h"
#include "call_buffers.h"
#include "inla_internal.h"
#include "integrate_host.h"

using inla::set_last_error;
namespace G = inla::integ;

namespace {

constexpr int kD = G::kD;
constexpr int kBatch = 256;                 // items per batched f call
constexpr size_t kLatentBytes = 1ull << 30; // mu and variances of one latent chunk

}  // namespace

extern "C" {

inla_status inla_integrate(const inla_model *model, const double *theta_mode,
                           const inla_integrate_opts *opts, inla_integrate_result *res,
                           double *points_or_null, int32_t points_cap, double *x_mean_dev,
                           double *x_var_dev, void *hip_stream) {
  set_last_error(INLA_OK, "");
  if (!model || !theta_mode || !res) return set_last_error(INLA_ERR_ARG, "need model, theta_mode and res");
  for (int k = 0; k < kD; ++k)
    if (!std::isfinite(theta_mode[k])) return set_last_error(INLA_ERR_ARG, "theta_mode is not finite");
  if (points_or_null && points_cap < 0) return set_last_error(INLA_ERR_ARG, "points_cap < 0");
  const double h = (opts && opts->h > 0.0) ? opts->h : 1e-3;
  const double dz = (opts && opts->dz > 0.0) ? opts->dz : 1.0;
  const double dpi = (opts && opts->dpi > 0.0) ? opts->dpi : 2.5;
  const int max_steps = (opts && opts->max_steps > 0) ? opts->max_steps : 6;
  const long long max_box = (opts && opts->max_box > 0) ? opts->max_box : 20000;
  const inla_opts *eo = opts ? opts->eval_opts : nullptr;
  if (max_steps > 64) return set_last_error(INLA_ERR_ARG, "max_steps above 64");
  if (!std::isfinite(h) || !std::isfinite(dz) || !std::isfinite(dpi))
    return set_last_error(INLA_ERR_ARG, "h, dz and dpi must be finite");
  int64_t n64 = 0;
  if (inla_model_shape(model, nullptr, nullptr, nullptr, &n64, nullptr) != INLA_OK)
    return set_last_error(INLA_ERR_ARG, "invalid model");
  const long long n = n64;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  std::memset(res, 0, sizeof(*res));

  inla::CallBuffers bufs;
  const int cap = std::max(kBatch, 2 * kD * max_steps);
  double *d_th = nullptr, *d_f = nullptr, *d_g = nullptr;
  int *d_st = nullptr;
  if (!bufs.get(&d_th, (size_t)cap * kD) || !bufs.get(&d_f, cap) ||
      !bufs.get(&d_g, (size_t)(2 * kD + 1) * kD) || !bufs.get(&d_st, cap))
    return set_last_error(INLA_ERR_NOMEM, "integration buffers");
  std::vector<const inla_model *> ms(cap, model);

  auto to_host = [&](void *dst, const void *src, size_t bytes) {
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s) == hipSuccess;
  };
  // f at a list of points (k x 4 host doubles) in batched calls; +inf where
  // the item's status is not 0
  auto eval_points = [&](const std::vector<double> &th, std::vector<double> &f) -> inla_status {
    const size_t K = th.size() / kD;
    f.assign(K, 0.0);
    std::vector<int> st(cap);
    for (size_t b0 = 0; b0 < K; b0 += cap) {
      const int k = (int)std::min<size_t>(cap, K - b0);
      if (hipMemcpyAsync(d_th, th.data() + b0 * kD, (size_t)k * kD * 8, hipMemcpyHostToDevice, s) != hipSuccess)
        return set_last_error(INLA_ERR_HIP, "integration copy to the device");
      const inla_status e = inla_eval_f(ms.data(), k, d_th, d_f, nullptr, nullptr, d_st, eo, s);
      if (e != INLA_OK) return e;
      if (!to_host(f.data() + b0, d_f, (size_t)k * 8) || !to_host(st.data(), d_st, (size_t)k * 4) ||
          hipStreamSynchronize(s) != hipSuccess)
        return set_last_error(INLA_ERR_HIP, "integration copy to the host");
      for (int i = 0; i < k; ++i)
        if (st[i] != 0 || !std::isfinite(f[b0 + i])) f[b0 + i] = std::numeric_limits<double>::infinity();
      res->f_evals += k;
    }
    return INLA_OK;
  };

  // 1. Hessian by central differences of the gradient: theta*, theta* + h e_k,
  //    theta* - h e_k in one batched call
  const int nh = 2 * kD + 1;
  std::vector<double> th(nh * kD);
  for (int i = 0; i < nh; ++i) {
    std::memcpy(&th[i * kD], theta_mode, kD * 8);
    if (i > 0) th[i * kD + (i - 1) % kD] += (i <= kD ? h : -h);
  }
  std::vector<double> fh(nh), gh(nh * kD);
  std::vector<int> sth(nh);
  {
    if (hipMemcpyAsync(d_th, th.data(), th.size() * 8, hipMemcpyHostToDevice, s) != hipSuccess)
      return set_last_error(INLA_ERR_HIP, "integration copy to the device");
    const inla_status e = inla_eval_f_grad(ms.data(), nh, d_th, d_f, d_g, nullptr, nullptr, d_st, eo, s);
    if (e != INLA_OK) return e;
    if (!to_host(fh.data(), d_f, nh * 8) || !to_host(gh.data(), d_g, gh.size() * 8) ||
        !to_host(sth.data(), d_st, nh * 4) || hipStreamSynchronize(s) != hipSuccess)
      return set_last_error(INLA_ERR_HIP, "integration copy to the host");
    res->grad_evals += nh;
    for (int i = 0; i < nh; ++i)
      if (sth[i] != 0 || !std::isfinite(fh[i]))
        return set_last_error(INLA_ERR_NOT_SPD, "f or its gradient cannot be evaluated at the mode stencil");
  }
  const double f0 = fh[0];
  res->f_mode = f0;
  for (int k = 0; k < kD; ++k) res->grad_mode[k] = gh[k];
  double H[kD][kD];
  for (int k = 0; k < kD; ++k)
    for (int j = 0; j < kD; ++j)
      H[k][j] = (gh[(1 + k) * kD + j] - gh[(1 + kD + k) * kD + j]) / (2.0 * h);
  for (int k = 0; k < kD; ++k)
    for (int j = k + 1; j < kD; ++j) H[k][j] = H[j][k] = 0.5 * (H[k][j] + H[j][k]);
  for (int k = 0; k < kD; ++k)
    for (int j = 0; j < kD; ++j) res->hessian[k * kD + j] = H[k][j];

  // 2. standardised coordinates
  double lam[kD], V[kD][kD], M[kD][kD];
  G::sym_eigen4(H, lam, V);
  for (int j = 0; j < kD; ++j) {
    res->eigval[j] = lam[j];
    for (int i = 0; i < kD; ++i) res->eigvec[i * kD + j] = V[i][j];
  }
  for (int j = 0; j < kD; ++j)
    if (!(lam[j] > 0.0)) return set_last_error(INLA_ERR_NOT_SPD, "the Hessian at theta_mode is not positive definite");
  for (int i = 0; i < kD; ++i)
    for (int j = 0; j < kD; ++j) M[i][j] = V[i][j] / std::sqrt(lam[j]);

  // 3. axis exploration: every step of every direction in one batched call
  std::vector<double> ax((size_t)2 * kD * max_steps * kD), fax;
  for (int j = 0; j < kD; ++j)
    for (int sg = 0; sg < 2; ++sg)
      for (int st = 1; st <= max_steps; ++st) {
        int sv[kD] = {0, 0, 0, 0};
        sv[j] = sg == 0 ? st : -st;
        G::theta_at(theta_mode, M, dz, sv, &ax[(((size_t)j * 2 + sg) * max_steps + (st - 1)) * kD]);
      }
  inla_status rc = eval_points(ax, fax);
  if (rc != INLA_OK) return rc;
  int lo[kD], hi[kD];
  for (int j = 0; j < kD; ++j)
    for (int sg = 0; sg < 2; ++sg) {
      int r = 0;
      for (int st = 1; st <= max_steps; ++st) {
        if (!(fax[((size_t)j * 2 + sg) * max_steps + (st - 1)] - f0 < dpi)) break;
        r = st;
      }
      (sg == 0 ? hi : lo)[j] = r;
    }
  for (int j = 0; j < kD; ++j) {
    res->lo[j] = lo[j];
    res->hi[j] = hi[j];
  }

  // 4. the box of candidates
  const long long nbox = G::box_size(lo, hi);
  if (nbox > max_box) return set_last_error(INLA_ERR_ARG, "the integration box holds more points than max_box");
  const std::vector<int> S = G::box_points(lo, hi);
  std::vector<double> bth((size_t)nbox * kD), fb;
  for (long long q = 0; q < nbox; ++q) G::theta_at(theta_mode, M, dz, &S[q * kD], &bth[q * kD]);
  rc = eval_points(bth, fb);
  if (rc != INLA_OK) return rc;
  res->n_box = (int)nbox;
  std::vector<long long> kept;
  std::vector<double> kf, kth;
  for (long long q = 0; q < nbox; ++q)
    if (fb[q] - f0 < dpi) {
      kept.push_back(q);
      kf.push_back(fb[q]);
      kth.insert(kth.end(), &bth[q * kD], &bth[q * kD] + kD);
    }
  const int K = (int)kept.size();
  res->n_points = K;
  if (K == 0) return set_last_error(INLA_ERR_NOT_SPD, "no grid point kept (f at the mode exceeds its neighbours)");

  // 5. quadrature over theta
  std::vector<double> w;
  double mean[kD], cov[kD][kD], log_ev = 0.0;
  G::quadrature(f0, kf, kth, lam, dz, w, mean, cov, log_ev);
  for (int i = 0; i < kD; ++i) {
    res->theta_mean[i] = mean[i];
    for (int j = 0; j < kD; ++j) res->theta_cov[i * kD + j] = cov[i][j];
  }
  res->log_evidence = log_ev;
  if (points_or_null)
    for (int k = 0; k < std::min(K, (int)points_cap); ++k) {
      double *row = points_or_null + (size_t)k * 10;
      for (int j = 0; j < kD; ++j) row[j] = S[kept[k] * kD + j];
      for (int j = 0; j < kD; ++j) row[kD + j] = kth[(size_t)k * kD + j];
      row[8] = kf[k];
      row[9] = w[k];
    }

  // 6. latent marginals: the mixture over the kept points, chunk by chunk
  if (!x_mean_dev && !x_var_dev) return INLA_OK;
  int chunk = (int)std::max<long long>(1, std::min<long long>(K, (long long)(kLatentBytes / (16ull * n))));
  // INLA_LATENT_CHUNK=c in the environment caps the points per chunk (the
  // chunks continue one sequential sum, so the results do not depend on it)
  if (const char *e = getenv("INLA_LATENT_CHUNK")) {
    const int c = atoi(e);
    if (c >= 1) chunk = std::min(chunk, c);
  }
  double *d_mu = nullptr, *d_var = nullptr, *d_shift = nullptr, *d_am = nullptr, *d_as = nullptr, *d_w = nullptr,
         *d_th2 = nullptr, *d_f2 = nullptr;
  int *d_st2 = nullptr;
  if (!bufs.get(&d_mu, (size_t)chunk * n) || !bufs.get(&d_var, (size_t)chunk * n) ||
      !bufs.get(&d_shift, n) || !bufs.get(&d_am, n) || !bufs.get(&d_as, n) || !bufs.get(&d_w, chunk) ||
      !bufs.get(&d_th2, (size_t)chunk * kD) || !bufs.get(&d_f2, chunk) || !bufs.get(&d_st2, chunk))
    return set_last_error(INLA_ERR_NOMEM, "latent mixture buffers");
  std::vector<const inla_model *> mk(chunk, model);
  std::vector<int> st2(chunk);
  // the shift: mu at the mode
  if (hipMemcpyAsync(d_th2, theta_mode, kD * 8, hipMemcpyHostToDevice, s) != hipSuccess)
    return set_last_error(INLA_ERR_HIP, "integration copy to the device");
  rc = inla_eval_f(mk.data(), 1, d_th2, d_f2, d_shift, nullptr, d_st2, eo, s);
  if (rc != INLA_OK) return rc;
  ++res->f_evals;
  for (int c0 = 0; c0 < K; c0 += chunk) {
    const int k = std::min(chunk, K - c0);
    if (hipMemcpyAsync(d_th2, &kth[(size_t)c0 * kD], (size_t)k * kD * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(d_w, &w[c0], (size_t)k * 8, hipMemcpyHostToDevice, s) != hipSuccess)
      return set_last_error(INLA_ERR_HIP, "integration copy to the device");
    rc = inla_eval_f(mk.data(), k, d_th2, d_f2, d_mu, d_var, d_st2, eo, s);
    if (rc != INLA_OK) return rc;
    res->f_evals += k;
    if (!to_host(st2.data(), d_st2, (size_t)k * 4) || hipStreamSynchronize(s) != hipSuccess)
      return set_last_error(INLA_ERR_HIP, "integration copy to the host");
    for (int i = 0; i < k; ++i)
      if (st2[i] != 0) return set_last_error(INLA_ERR_NOT_SPD, "a kept point failed its partial inversion");
    if (inla::launch_mixture_accumulate(d_mu, d_var, d_w, k, n, d_shift, d_am, d_as, c0 == 0 ? 1 : 0, s) !=
        hipSuccess)
      return set_last_error(INLA_ERR_HIP, "mixture kernel launch");
  }
  if (inla::launch_mixture_finish(d_shift, d_am, d_as, n, x_mean_dev, x_var_dev, s) != hipSuccess)
    return set_last_error(INLA_ERR_HIP, "mixture kernel launch");
  if (hipStreamSynchronize(s) != hipSuccess) return set_last_error(INLA_ERR_HIP, "integration synchronise");
  return INLA_OK;
}

}  // extern "C"
