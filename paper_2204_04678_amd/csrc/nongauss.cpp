// f(theta) and its exact gradient with a Poisson likelihood (paper, Sec.
// "Latent Gaussian Models": with a non-Gaussian likelihood the Gaussian
// approximation of eq. (post_theta_approx) is found by an inner optimisation,
// its mode and normalising constant anew in every iteration).
//
// The inner loop is Newton's method on the mode: in every iteration the
// precision Q_c(x) = Q_p + A^T diag(exp(A x)) A is assembled (the prior
// blocks plus the observation terms of the current x) and factored, and
// Q_c(x) x_new = A^T (y + e (eta - 1)) is solved; the step is halved until
// the objective log pi(x | theta) + log pi(y | x) does not decrease.  At the
// mode x*, f = -log pi(theta) - 1/2 log|Q_p| + 1/2 x*^T Q_p x*
// - log pi(y | x*) + 1/2 log|Q_c(x*)|, and
//   df/dtheta_k = p_k (theta_k - m_k) - 1/2 tr(Q_p^{-1} dQ_k) + 1/2 x*^T dQ_k x*
//                 + 1/2 tr(Q_c^{-1} dQ_k) - z^T dQ_k x*,
// z = Q_c^{-1} A^T c, c_i = 1/2 exp(eta_i) (A Q_c^{-1} A^T)_ii (derived: the
// mode moves with theta, dx*/dtheta_k = -Q_c^{-1} dQ_k x*, and log|Q_c|
// depends on x*).  The traces and the (A Q_c^{-1} A^T)_ii come from the
// selected inverses of both factors; every step is a kernel of the library,
// the host only steers the iteration and adds up a handful of scalars.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/inla_bta.h"
#include "call_buffers.h"
#include "inla_internal.h"

using inla::set_last_error;

namespace {

// the storage of one BTA matrix of the model's shape
bool bta_buffers(inla::CallBuffers &B, inla_bta &q, int b, int nt, int a) {
  q.b = b; q.nt = nt; q.a = a;
  q.S = nullptr; q.R = nullptr; q.T = nullptr;
  if (!B.get(&q.D, (size_t)nt * b * b)) return false;
  if (nt > 1 && !B.get(&q.S, (size_t)(nt - 1) * b * b)) return false;
  if (a > 0 && (!B.get(&q.R, (size_t)nt * a * b) || !B.get(&q.T, (size_t)a * a))) return false;
  return true;
}

}  // namespace

extern "C" {

inla_status inla_eval_f_grad_poisson(const inla_model *model, const double *theta,
                                     const inla_newton_opts *opts, inla_newton_result *res,
                                     double *x_mode_dev, double *var_dev, void *hip_stream) {
  set_last_error(INLA_OK, "");
  if (!model || !theta || !res) return set_last_error(INLA_ERR_ARG, "need model, theta and res");
  for (int k = 0; k < 4; ++k)
    if (!std::isfinite(theta[k])) return set_last_error(INLA_ERR_ARG, "theta is not finite");
  if (!(std::fabs(std::tanh(theta[2])) < 1.0)) return set_last_error(INLA_ERR_ARG, "tanh(theta_3) = +-1");
  double log_y_fact = 0.0;
  if (!inla::model_counts(model, &log_y_fact))
    return set_last_error(INLA_ERR_ARG, "the model's responses are not counts (non-negative integers)");
  const int max_iter = (opts && opts->max_iter > 0) ? opts->max_iter : 100;
  const double tol = (opts && opts->tol > 0.0) ? opts->tol : 1e-12;
  const bool warm = opts && opts->warm != 0;
  if (warm && !x_mode_dev) return set_last_error(INLA_ERR_ARG, "warm start needs x_mode_dev");
  const inla::ModelDev &H = inla::model_host_desc(model);
  const inla::ModelDev *Md = inla::model_device(model);
  const int b = H.b, nt = H.nt, a = H.a;
  const long long n = H.n, m = H.m;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  std::memset(res, 0, sizeof(*res));
  res->f = NAN;
  for (double &g : res->grad) g = NAN;

  inla::CallBuffers B;
  inla_bta Qp, Qc, Sg;
  double *th, *x, *xn, *cand, *e, *w, *rhs, *c, *z, *part, *ld;
  int *info;
  if (!bta_buffers(B, Qp, b, nt, a) || !bta_buffers(B, Qc, b, nt, a) || !bta_buffers(B, Sg, b, nt, a) || !B.get(&th, 4) ||
      !B.get(&x, n) || !B.get(&xn, n) || !B.get(&cand, n) || !B.get(&e, m) || !B.get(&w, m) ||
      !B.get(&rhs, n) || !B.get(&c, m) || !B.get(&z, n) || !B.get(&part, 4 * inla::kNgBlocks) ||
      !B.get(&ld, 2) || !B.get(&info, 2))
    return set_last_error(INLA_ERR_NOMEM, "Poisson evaluation buffers");
  std::vector<double> hp(4 * inla::kNgBlocks);

#define NG_HIP(expr, what)                                                  \
  do {                                                                      \
    if ((expr) != hipSuccess) return set_last_error(INLA_ERR_HIP, what);   \
  } while (0)
#define NG_TRY(expr)                     \
  do {                                   \
    const inla_status st_ = (expr);      \
    if (st_ != INLA_OK) return st_;      \
  } while (0)

  // partial sums of a kernel, added on the host in block order
  auto sums = [&](int width, double *out) -> bool {
    if (hipMemcpyAsync(hp.data(), part, (size_t)width * inla::kNgBlocks * 8, hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return false;
    for (int k = 0; k < width; ++k) out[k] = 0.0;
    for (int blk = 0; blk < inla::kNgBlocks; ++blk)
      for (int k = 0; k < width; ++k) out[k] += hp[(size_t)blk * width + k];
    return true;
  };
  // log pi(y | v) + sum log y! and v^T Q_p v
  auto loglik = [&](const double *v, double *eo, double *wo, double &ll) -> bool {
    if (inla::launch_ng_obs(Md, m, v, eo, wo, part, s) != hipSuccess) return false;
    return sums(1, &ll);
  };
  auto quad = [&](const double *u, const double *v, double q[4]) -> bool {
    if (inla::launch_ng_quad(Md, th, u, v, part, s) != hipSuccess) return false;
    return sums(4, q);
  };
  auto objective = [&](const double *v, double &g) -> bool {
    double ll = 0.0, q[4];
    if (!loglik(v, nullptr, nullptr, ll) || !quad(v, v, q)) return false;
    g = -0.5 * (q[0] + H.beta_prec * q[3]) + ll;
    return true;
  };
  // Q_c(v) = Q_p + A^T diag(e(v)) A into Qc, factored; e must hold exp(A v)
  auto factor_qc = [&](double *ld_dev, int *info_dev) -> inla_status {
    NG_TRY(inla_assemble(model, th, 0, &Qc, nullptr, s));
    NG_HIP(inla::launch_ng_add_obs(Md, b, nt, a, H.nnz, e, Qc.D, Qc.R, Qc.T, s), "observation terms");
    return inla_factor_logdet(&Qc, ld_dev, info_dev, s);
  };
  auto read_info = [&](const int *info_dev, int &v) -> bool {
    return hipMemcpyAsync(&v, info_dev, 4, hipMemcpyDeviceToHost, s) == hipSuccess &&
           hipStreamSynchronize(s) == hipSuccess;
  };

  NG_HIP(hipMemcpyAsync(th, theta, 32, hipMemcpyHostToDevice, s), "theta to the device");
  // Q_p and its factor
  NG_TRY(inla_assemble(model, th, 0, &Qp, nullptr, s));
  NG_TRY(inla_factor_logdet(&Qp, ld, info, s));
  int inf = 0;
  NG_HIP(read_info(info, inf) ? hipSuccess : hipErrorUnknown, "factor status");
  if (inf != 0) {
    res->status = 1;
    return INLA_OK;
  }

  // Newton's method on the mode
  if (warm) NG_HIP(hipMemcpyAsync(x, x_mode_dev, (size_t)n * 8, hipMemcpyDeviceToDevice, s), "warm start");
  else NG_HIP(inla::launch_fill(x, n, 0.0, s), "start");
  double gx = 0.0;
  NG_HIP(objective(x, gx) ? hipSuccess : hipErrorUnknown, "objective");
  bool converged = false;
  for (int it = 1; it <= max_iter && !converged; ++it) {
    double ll = 0.0;
    NG_HIP(loglik(x, e, w, ll) ? hipSuccess : hipErrorUnknown, "observation pass");
    NG_TRY(factor_qc(ld + 1, info + 1));
    NG_HIP(read_info(info + 1, inf) ? hipSuccess : hipErrorUnknown, "factor status");
    if (inf != 0) {
      res->status = 2;
      res->iterations = it;
      return INLA_OK;
    }
    NG_HIP(inla::launch_ng_atv(Md, (long long)b * nt, a, w, rhs, s), "A^T w");
    NG_TRY(inla_solve(&Qc, rhs, xn, 1, s));
    double step = 1.0, gc = 0.0, mx[2] = {0.0, 0.0};
    for (int h = 0;; ++h) {
      NG_HIP(inla::launch_ng_step(x, xn, step, cand, n, part, s), "step");
      NG_HIP(hipMemcpyAsync(hp.data(), part, 2 * inla::kNgBlocks * 8, hipMemcpyDeviceToHost, s), "step");
      NG_HIP(hipStreamSynchronize(s), "step");
      mx[0] = mx[1] = 0.0;
      for (int blk = 0; blk < inla::kNgBlocks; ++blk) {
        mx[0] = std::max(mx[0], hp[2 * blk]);
        mx[1] = std::max(mx[1], hp[2 * blk + 1]);
      }
      NG_HIP(objective(cand, gc) ? hipSuccess : hipErrorUnknown, "objective");
      if (gc >= gx) break;
      if (h >= 60) {
        // no step along the Newton direction keeps the objective (a NaN from
        // an overflowing exp(eta), say): no mode, rather than a tiny step
        // taken for convergence
        res->status = 4;
        res->iterations = it;
        return INLA_OK;
      }
      step *= 0.5;
      ++res->halvings;
    }
    NG_HIP(hipMemcpyAsync(x, cand, (size_t)n * 8, hipMemcpyDeviceToDevice, s), "iterate");
    gx = gc;
    res->iterations = it;
    converged = mx[0] <= tol * (1.0 + mx[1]);
  }
  if (!converged) {
    res->status = 4;
    return INLA_OK;
  }

  // at the mode: Q_c(x*), its log-determinant, the likelihood and x*^T Q_p x*
  double ll = 0.0, qxx[4];
  NG_HIP(loglik(x, e, nullptr, ll) ? hipSuccess : hipErrorUnknown, "observation pass");
  NG_TRY(factor_qc(ld + 1, info + 1));
  NG_HIP(read_info(info + 1, inf) ? hipSuccess : hipErrorUnknown, "factor status");
  if (inf != 0) {
    res->status = 2;
    return INLA_OK;
  }
  NG_HIP(quad(x, x, qxx) ? hipSuccess : hipErrorUnknown, "quadratic forms");
  double lds[2];
  NG_HIP(hipMemcpyAsync(lds, ld, 16, hipMemcpyDeviceToHost, s), "log-determinants");
  NG_HIP(hipStreamSynchronize(s), "log-determinants");
  double lp = 0.0;
  for (int k = 0; k < 4; ++k) {
    const double dv = theta[k] - H.prior_mean[k];
    lp += 0.5 * std::log(H.prior_prec[k] / (2.0 * 3.14159265358979323846)) - 0.5 * H.prior_prec[k] * dv * dv;
  }
  res->logdet_p = lds[0];
  res->logdet_c = lds[1];
  res->log_lik = ll - log_y_fact;
  res->quad = qxx[0] + H.beta_prec * qxx[3];
  res->f = -lp - 0.5 * lds[0] + 0.5 * res->quad - res->log_lik + 0.5 * lds[1];

  // traces tr(Sigma dQ_k) of both selected inverses through the library's
  // trace kernel (an item whose Sigma blocks are the caller-layout ones)
  std::vector<double> trp((size_t)(nt + 1) * inla::kTraceBlocks * 4);
  double *trd;
  inla::ItemDev *itd;
  if (!B.get(&trd, trp.size()) || !B.get(&itd, 1)) return set_last_error(INLA_ERR_NOMEM, "trace buffers");
  auto traces = [&](inla_bta &L, double *diag, double tr[4]) -> inla_status {
    NG_TRY(inla_selinv(&L, &Sg, nullptr, s));
    inla::ItemDev it;
    std::memset(&it, 0, sizeof(it));
    it.b = b; it.nt = nt; it.a = a; it.nP = (b + inla::kTile - 1) / inla::kTile;
    it.ntf = nt; it.trev = 0; it.nrun = nt; it.own_arrow = 1; it.sbw = b;
    it.SD = Sg.D; it.sd_stride = (long long)b * b;
    it.SS = Sg.S; it.ss_stride = (long long)b * b;
    it.SR = Sg.R; it.sr_stride = (long long)a * b;
    it.ST = Sg.T;
    it.trpart = trd; it.diag = diag; it.model = Md; it.theta = th; it.which = 0;
    NG_HIP(hipMemcpyAsync(itd, &it, sizeof(it), hipMemcpyHostToDevice, s), "trace descriptor");
    for (int t = -1; t < nt; ++t) NG_HIP(inla::launch_trace_step(itd, 1, t, s), "traces");
    NG_HIP(hipMemcpyAsync(trp.data(), trd, trp.size() * 8, hipMemcpyDeviceToHost, s), "traces");
    NG_HIP(hipStreamSynchronize(s), "traces");
    for (int k = 0; k < 4; ++k) tr[k] = 0.0;
    for (size_t q = 0; q < trp.size(); q += 4)
      for (int k = 0; k < 4; ++k) tr[k] += trp[q + k];
    return INLA_OK;
  };
  double trP[4], trC[4];
  NG_TRY(traces(Qp, nullptr, trP));
  NG_TRY(traces(Qc, var_dev, trC));
  // the implicit term: c_i = 1/2 e_i (A Sigma_c A^T)_ii, z = Q_c^{-1} A^T c
  NG_HIP(inla::launch_ng_obs_var(Md, m, Sg.D, Sg.R, Sg.T, e, c, s), "observation variances");
  NG_HIP(inla::launch_ng_atv(Md, (long long)b * nt, a, c, rhs, s), "A^T c");
  NG_TRY(inla_solve(&Qc, rhs, z, 1, s));
  double qzx[4];
  NG_HIP(quad(z, x, qzx) ? hipSuccess : hipErrorUnknown, "quadratic forms");
  // d/dtheta_1 of Q_st is 2 Q_st; the fixed effects' prior does not move
  const double dxx[3] = {2.0 * qxx[0], qxx[1], qxx[2]};
  const double dzx[3] = {2.0 * qzx[0], qzx[1], qzx[2]};
  for (int k = 0; k < 4; ++k) res->grad[k] = H.prior_prec[k] * (theta[k] - H.prior_mean[k]);
  for (int k = 0; k < 3; ++k)
    res->grad[k] += -0.5 * trP[k] + 0.5 * dxx[k] + 0.5 * trC[k] - dzx[k];
  if (x_mode_dev) NG_HIP(hipMemcpyAsync(x_mode_dev, x, (size_t)n * 8, hipMemcpyDeviceToDevice, s), "mode out");
  NG_HIP(hipStreamSynchronize(s), "synchronise");
  res->status = 0;
  return INLA_OK;
#undef NG_HIP
#undef NG_TRY
}

}  // extern "C"
