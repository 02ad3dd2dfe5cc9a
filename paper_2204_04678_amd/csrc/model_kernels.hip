// Model-specific kernels: assembly of the BTA precision blocks, the block
// substitution sweeps, the trace reductions of the selected inverse against
// the derivative blocks, the posterior-mode terms and the final combination
// of f(theta) and its gradient.
//
// Model (paper, Sec. "Latent Gaussian Models", latent vector without the
// linear predictor): x = (u_0..u_{nt-1}, beta) is Gaussian with precision
//   Q_prior = blockdiag(Q_AR1(rho) (x) Q_s(tau, kappa), beta_prec I),
//   Q_s = (tau^2 / h^2) (kappa^2 h^2 I + G)^2,
//   Q_AR1 = T(rho) / (1 - rho^2)  (stationary AR1, unit marginal variance),
// observations y = A x + e, e ~ N(0, tau_y^{-1} I), so that
//   Q_c = Q_prior + tau_y A^T A and the mode solves Q_c mu = tau_y A^T y.
#include <algorithm>
#include <cmath>

#include "inla_internal.h"

namespace inla {

namespace {

struct Coef {
  double tau, kappa, rho, tauy;
  double qsc;    // tau^2 / h^2
  double k2;     // kappa^2 h^2
  double dq2;    // 4 tau^2 kappa^2  (d Q_s / d log kappa = dq2 (k2 I + G))
  double inv1mr2;
};

__device__ inline Coef make_coef(const ModelDev &M, const double *th) {
  Coef c;
  c.tau = exp(th[0]);
  c.kappa = exp(th[1]);
  c.rho = tanh(th[2]);
  c.tauy = exp(th[3]);
  c.qsc = c.tau * c.tau / (M.h * M.h);
  c.k2 = c.kappa * c.kappa * M.h * M.h;
  c.dq2 = 4.0 * c.tau * c.tau * c.kappa * c.kappa;
  c.inv1mr2 = 1.0 / (1.0 - c.rho * c.rho);
  return c;
}

// AR1 precision entries and their theta_3 derivatives (rho = tanh theta_3).
__device__ inline double ar1_diag(const Coef &c, int t, int nt) {
  if (nt == 1) return 1.0;
  return (t == 0 || t == nt - 1) ? c.inv1mr2 : (1.0 + c.rho * c.rho) * c.inv1mr2;
}
__device__ inline double ar1_off(const Coef &c) { return -c.rho * c.inv1mr2; }
__device__ inline double ar1_ddiag(const Coef &c, int t, int nt) {
  if (nt == 1) return 0.0;
  return (t == 0 || t == nt - 1) ? 2.0 * c.rho * c.inv1mr2 : 4.0 * c.rho * c.inv1mr2;
}
__device__ inline double ar1_doff(const Coef &c) { return -(1.0 + c.rho * c.rho) * c.inv1mr2; }

// Q_s and dQ_s/dtheta_2 on pattern entry e.
__device__ inline double qs_entry(const ModelDev &M, const Coef &c, int e) {
  return c.qsc * (c.k2 * c.k2 * M.pdelta[e] + 2.0 * c.k2 * M.pg1[e] + M.pg2[e]);
}
__device__ inline double dqs_entry(const ModelDev &M, const Coef &c, int e) {
  return c.dq2 * (c.k2 * M.pdelta[e] + M.pg1[e]);
}

template <int NT>
__device__ inline void block_reduce(double (&v)[4], double *red) {
  // fixed-order tree over the workgroup; result in red[0..3]
  const int tid = threadIdx.x;
#pragma unroll
  for (int k = 0; k < 4; ++k) red[k * NT + tid] = v[k];
  __syncthreads();
  for (int off = NT / 2; off > 0; off >>= 1) {
    if (tid < off) {
#pragma unroll
      for (int k = 0; k < 4; ++k) red[k * NT + tid] += red[k * NT + tid + off];
    }
    __syncthreads();
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// assembly
// ---------------------------------------------------------------------------

// Each workgroup writes kAsmCols columns of one b x b block (D[t] for
// blockIdx.y < nt, S[t] for blockIdx.y - nt).  A column is built in LDS, in
// pieces of kAsmRows rows: zeros, then the pattern's entries scattered to
// their rows (distinct within a column), then one coalesced store; entries
// outside the pattern are zero.
constexpr int kAsmCols = 4;
constexpr int kAsmRows = 2048;
__global__ __launch_bounds__(256) void assemble_blocks_kernel(const ModelDev *__restrict__ Mp,
                                                              const double *theta, int which,
                                                              double *D, double *S) {
  __shared__ double piece[kAsmRows];
  const ModelDev &M = *Mp;
  const int b = M.b, nt = M.nt;
  const int blk = blockIdx.y;
  const bool isS = blk >= nt;
  const int t = isS ? blk - nt : blk;
  const Coef c = make_coef(M, theta);
  const double cblk = isS ? ar1_off(c) : ar1_diag(c, t, nt);
  const bool add_obs = !isS && which;
  for (int s = blockIdx.x * kAsmCols; s < min(b, (blockIdx.x + 1) * kAsmCols); ++s) {
    double *col = (isS ? S : D) + (long long)t * b * b + (long long)s * b;
    const int e0 = M.colptr[s], e1 = M.colptr[s + 1];
    for (int r0 = 0; r0 < b; r0 += kAsmRows) {
      const int rn = min(kAsmRows, b - r0);
      for (int i = threadIdx.x; i < rn; i += blockDim.x) piece[i] = 0.0;
      __syncthreads();
      for (int e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
        const int i = M.rowidx[e] - r0;
        if (i >= 0 && i < rn) {
          double v = cblk * qs_entry(M, c, e);
          if (add_obs) v += c.tauy * M.AtA[(long long)t * M.nnz + e];
          piece[i] = v;
        }
      }
      __syncthreads();
      for (int i = threadIdx.x; i < rn; i += blockDim.x) col[r0 + i] = piece[i];
      __syncthreads();
    }
  }
}

// Arrow blocks: R[t] = tau_y (Z^T A_t) (Q_c) or 0; T = beta_prec I (+ tau_y Z^T Z);
// rhs = tau_y A^T y.
__global__ void assemble_arrow_kernel(const ModelDev *__restrict__ Mp, const double *theta, int which,
                                      double *R, double *T, double *rhs) {
  const ModelDev &M = *Mp;
  const int a = M.a;
  const long long nR = (long long)M.nt * a * M.b;
  const long long nT = (long long)a * a;
  const long long nrhs = rhs ? M.n : 0;
  const double tauy = exp(theta[3]);
  const long long total = nR + nT + nrhs;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    if (i < nR) {
      R[i] = which ? tauy * M.ZtA[i] : 0.0;
    } else if (i < nR + nT) {
      const long long k = i - nR;
      const int r = (int)(k % a), cc = (int)(k / a);
      T[k] = (r == cc ? M.beta_prec : 0.0) + (which ? tauy * M.ZtZ[k] : 0.0);
    } else {
      const long long k = i - nR - nT;
      rhs[k] = tauy * M.Aty[k];
    }
  }
}

hipError_t launch_assemble(const ModelDev *model_dev, int b, int nt, int a, const double *theta,
                           int which, double *D, double *S, double *R, double *T, double *rhs,
                           hipStream_t s) {
  hipLaunchKernelGGL(assemble_blocks_kernel, dim3((b + kAsmCols - 1) / kAsmCols, 2 * nt - 1),
                     dim3(256), 0, s, model_dev, theta, which, D, S);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const long long total = (long long)nt * a * b + (long long)a * a + (rhs ? (long long)b * nt + a : 0);
  if (total > 0) {
    const long long blocks = std::min<long long>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(assemble_arrow_kernel, dim3((unsigned)blocks), dim3(256), 0, s, model_dev,
                       theta, which, R, T, rhs);
    e = hipGetLastError();
  }
  return e;
}

// ---------------------------------------------------------------------------
// substitution sweeps with the inverse-diagonal factor
//   forward:  z_t = Linv_tt (r_t - L_{t,t-1} z_{t-1}),  z_A = Linv_AA (r_A - sum_t L_{A,t} z_t)
//   backward: x_A = Linv_AA^T z_A,  x_t = Linv_tt^T (z_t - L_{t+1,t}^T x_{t+1} - L_{A,t}^T x_A)
// ---------------------------------------------------------------------------

__global__ void solve_stage_kernel(const ItemDev *__restrict__ items, int t, int stage,
                                   double *const *xs, double *const *tmps) {
  const ItemDev it = items[blockIdx.y];
  const int b = it.b, a = it.a, nt = it.nt;
  const long long bb = (long long)b * b;
  double *x = xs[blockIdx.y];
  double *tmp = tmps[blockIdx.y];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  __shared__ double red[4][64];
  __shared__ double xa[kMaxArrow];
  switch (stage) {
    case SV_F1:
    case SV_F2: {
      // 8 rows per workgroup, 32 column lanes per row (columns cl, cl + 32, ...);
      // the 32 partial sums of a row are added in a fixed order
      // (a backward chain runs its first stage at its last block, the middle
      // block of the matrix, which the forward chain factors: there it only
      // subtracts its coupling term from the middle block's right-hand side)
      if (t >= nt || (stage == SV_F2 && t >= it.nrun)) return;
      const int rr = tid & 7, cl = tid >> 3;
      const int r = blockIdx.x * 8 + rr;
      const double *M = (stage == SV_F1) ? (t > 0 ? sblk(it, t - 1) : nullptr) : dblk(it, t);
      const double *v = (stage == SV_F1) ? (t > 0 ? x + (long long)tmap(it, t - 1) * b : nullptr) : tmp;
      const int jend = (stage == SV_F1) ? b : min(b, blockIdx.x * 8 + 8);
      // four independent partial sums per lane keep four loads in flight
      double acc = 0.0;
      if (M && r < b) {
        double a4[4] = {0.0, 0.0, 0.0, 0.0};
        int j = cl;
        for (; j + 96 < jend; j += 128) {
#pragma unroll
          for (int u = 0; u < 4; ++u) a4[u] = fma(M[r + (long long)(j + 32 * u) * b], v[j + 32 * u], a4[u]);
        }
        for (; j < jend; j += 32) a4[0] = fma(M[r + (long long)j * b], v[j], a4[0]);
        acc = (a4[0] + a4[1]) + (a4[2] + a4[3]);
      }
      double *red8 = &red[0][0];   // [32][8]
      red8[cl * 8 + rr] = acc;
      __syncthreads();
      if (cl == 0 && r < b) {
        double sum = 0.0;
        for (int c = 0; c < 32; ++c) sum += red8[c * 8 + rr];
        double *xt = x + (long long)tmap(it, t) * b;
        if (stage == SV_F1) {
          if (t == it.nrun) xt[r] -= sum;
          else tmp[r] = xt[r] - sum;
        } else {
          xt[r] = sum;
        }
      }
      return;
    }
    case SV_FA1: {
      const int c = blockIdx.x;
      if (c >= a) return;
      const long long len = (long long)nt * b;
      double acc = 0.0;
      for (long long k = tid; k < len; k += blockDim.x) acc += it.R[c + k * a] * x[k];
      __shared__ double r1[256];
      r1[tid] = acc;
      __syncthreads();
      for (int off = 128; off > 0; off >>= 1) {
        if (tid < off) r1[tid] += r1[tid + off];
        __syncthreads();
      }
      if (tid == 0) tmp[c] = x[len + c] - r1[0];
      return;
    }
    case SV_FA2: {
      if (blockIdx.x != 0 || a == 0) return;
      if (tid < a) {
        double acc = 0.0;
        for (int j = 0; j <= tid; ++j) acc += it.T[tid + (long long)j * a] * tmp[j];
        x[(long long)nt * b + tid] = acc;
      }
      return;
    }
    case SV_BA: {
      if (blockIdx.x != 0 || a == 0) return;
      if (tid < a) xa[tid] = x[(long long)nt * b + tid];
      __syncthreads();
      if (tid < a) {
        double acc = 0.0;
        for (int i = tid; i < a; ++i) acc += it.T[i + (long long)tid * a] * xa[i];
        x[(long long)nt * b + tid] = acc;
      }
      return;
    }
    case SV_B1:
    case SV_B2: {
      if (t >= it.nrun) return;
      const int j = blockIdx.x * 4 + w;
      if (j >= b) return;
      double acc = 0.0;
      if (stage == SV_B1) {
        if (t < nt - 1) {
          const double *X = sblk(it, t) + (long long)j * b;
          const double *xn = x + (long long)tmap(it, t + 1) * b;
          // four independent partial sums keep four loads in flight
          double a4[4] = {0.0, 0.0, 0.0, 0.0};
          int i = lane;
          for (; i + 192 < b; i += 256) {
#pragma unroll
            for (int u = 0; u < 4; ++u) a4[u] = fma(X[i + 64 * u], xn[i + 64 * u], a4[u]);
          }
          for (; i < b; i += 64) a4[0] = fma(X[i], xn[i], a4[0]);
          acc = (a4[0] + a4[1]) + (a4[2] + a4[3]);
        }
        if (a > 0) {
          const double *Rt = rblk(it, t) + (long long)j * a;
          const double *xA = x + (long long)it.ntf * b;
          for (int c = lane; c < a; c += 64) acc += Rt[c] * xA[c];
        }
      } else {
        const double *L = dblk(it, t) + (long long)j * b;
        double a4[4] = {0.0, 0.0, 0.0, 0.0};
        int i = j + lane;
        for (; i + 192 < b; i += 256) {
#pragma unroll
          for (int u = 0; u < 4; ++u) a4[u] = fma(L[i + 64 * u], tmp[i + 64 * u], a4[u]);
        }
        for (; i < b; i += 64) a4[0] = fma(L[i], tmp[i], a4[0]);
        acc = (a4[0] + a4[1]) + (a4[2] + a4[3]);
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
      if (lane == 0) {
        double *xt = x + (long long)tmap(it, t) * b;
        if (stage == SV_B1) tmp[j] = xt[j] - acc;
        else xt[j] = acc;
      }
      return;
    }
    default:
      return;
  }
}

hipError_t launch_solve_stage(const ItemDev *items_dev, int n_items, int max_b, int max_a, int t,
                              int stage, double *const *xs_dev, double *const *tmps_dev,
                              hipStream_t s) {
  int gx = 1;
  switch (stage) {
    case SV_F1: case SV_F2: gx = (max_b + 7) / 8; break;
    case SV_B1: case SV_B2: gx = (max_b + 3) / 4; break;
    case SV_FA1: gx = max_a; break;
    default: gx = 1;
  }
  if (gx <= 0 || n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(solve_stage_kernel, dim3(gx, n_items), dim3(256), 0, s, items_dev, t, stage,
                     xs_dev, tmps_dev);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// traces tr(Sigma dQ/dtheta_k) over the BTA pattern, and marginal variances
// ---------------------------------------------------------------------------

// Per step t (t = -1: the arrow block) and item, kTraceBlocks workgroups each
// reduce a strided share of the pattern entries; workgroup k writes its four
// partial traces to trpart[(step * kTraceBlocks + k) * 4 ..] with step = t
// (t >= 0) or nt (arrow), and the combination adds them in a fixed order.
__global__ __launch_bounds__(256) void trace_step_kernel(const ItemDev *__restrict__ items, int t) {
  const ItemDev it = items[blockIdx.y];
  if (!it.trpart && !it.diag) return;
  const int b = it.b, a = it.a, nt = it.nt;
  const int tid = threadIdx.x, blk = blockIdx.x;
  const int g0 = blk * 256 + tid, gs = kTraceBlocks * 256;
  __shared__ double red[4 * 256];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  if (t < 0) {
    // arrow block: Sigma_T (a whole matrix only)
    if (!it.own_arrow) return;
    if (a > 0) {
      if (it.diag && blk == 0 && tid < a) it.diag[(long long)nt * b + tid] = it.ST[tid + (long long)tid * a];
      if (it.trpart && it.which == 1 && it.model) {
        const double tauy = exp(it.theta[3]);
        for (int k = g0; k < a * a; k += gs) v[3] += tauy * it.model->ZtZ[k] * it.ST[k];
      }
    }
    if (!it.trpart) return;
    block_reduce<256>(v, red);
    if (tid == 0) {
#pragma unroll
      for (int k = 0; k < 4; ++k) it.trpart[((long long)nt * kTraceBlocks + blk) * 4 + k] = red[k * 256];
    }
    return;
  }
  if (t >= it.nrun) return;
  const int tau = tmap(it, t);   // the time block of chain step t
  const double *SD = sig_D(it, t);
  if (it.diag) {
    for (int s = g0; s < b; s += gs) it.diag[(long long)tau * b + s] = SD[s + (long long)s * b];
  }
  if (!it.trpart) return;
  const ModelDev &M = *it.model;
  const Coef c = make_coef(M, it.theta);
  const double cD = ar1_diag(c, tau, it.ntf), cS = ar1_off(c);
  const double dcD = ar1_ddiag(c, tau, it.ntf), dcS = ar1_doff(c);
  const bool hasS = t < nt - 1;
  const double *SS = hasS ? sig_S(it, t) : nullptr;
  for (int e = g0; e < M.nnz; e += gs) {
    const int i = M.rowidx[e], s = M.colidx[e];
    const double q = qs_entry(M, c, e), dq = dqs_entry(M, c, e);
    const double sd = SD[i + (long long)s * b];
    v[0] += 2.0 * cD * q * sd;
    v[1] += cD * dq * sd;
    v[2] += dcD * q * sd;
    if (it.which == 1) v[3] += c.tauy * M.AtA[(long long)tau * M.nnz + e] * sd;
    if (hasS) {
      const double ss = SS[i + (long long)s * b];
      v[0] += 4.0 * cS * q * ss;
      v[1] += 2.0 * cS * dq * ss;
      v[2] += 2.0 * dcS * q * ss;
    }
  }
  if (it.which == 1 && a > 0) {
    const double *SR = sig_R(it, t);
    const double *Z = M.ZtA + (long long)tau * a * b;
    for (int k = g0; k < a * b; k += gs) v[3] += 2.0 * c.tauy * Z[k] * SR[k];
  }
  block_reduce<256>(v, red);
  if (tid == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) it.trpart[((long long)t * kTraceBlocks + blk) * 4 + k] = red[k * 256];
  }
}

hipError_t launch_trace_step(const ItemDev *items_dev, int n_items, int t, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(trace_step_kernel, dim3(kTraceBlocks, n_items), dim3(256), 0, s, items_dev, t);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// posterior-mode terms
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void terms_kernel(const TermItem *__restrict__ items) {
  const TermItem ti = items[blockIdx.y];
  const ModelDev &M = *ti.model;
  const int b = M.b, nt = M.nt;
  const Coef c = make_coef(M, ti.theta);
  const double cS = ar1_off(c), dcS = ar1_doff(c);
  const double *mu = ti.mu;
  const long long nst = (long long)nt * b;
  const long long stride = (long long)gridDim.x * blockDim.x;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < nst; idx += stride) {
    const int t = (int)(idx / b), s = (int)(idx % b);
    const double *mt = mu + (long long)t * b;
    const double *mn = (t < nt - 1) ? mt + b : nullptr;
    double q0 = 0.0, d0 = 0.0, q1 = 0.0, d1 = 0.0;
    for (int e = M.colptr[s]; e < M.colptr[s + 1]; ++e) {
      const int i = M.rowidx[e];
      const double q = qs_entry(M, c, e), dq = dqs_entry(M, c, e);
      q0 += q * mt[i];
      d0 += dq * mt[i];
      if (mn) {
        q1 += q * mn[i];
        d1 += dq * mn[i];
      }
    }
    const double u = mt[s];
    const double cD = ar1_diag(c, t, nt), dcD = ar1_ddiag(c, t, nt);
    v[0] += u * (cD * q0 + 2.0 * cS * q1);
    v[1] += u * (cD * d0 + 2.0 * cS * d1);
    v[2] += u * (dcD * q0 + 2.0 * dcS * q1);
  }
  for (long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x; j < M.m; j += stride) {
    double r = M.y[j];
    for (long long e = M.A_rowptr[j]; e < M.A_rowptr[j + 1]; ++e) r -= M.A_val[e] * mu[M.A_col[e]];
    v[3] += r * r;
  }
  __shared__ double red[4 * 256];
  block_reduce<256>(v, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) ti.part[(long long)blockIdx.x * 4 + k] = red[k * 256];
  }
}

hipError_t launch_terms(const TermItem *items_dev, int n_items, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(terms_kernel, dim3(kTermBlocks, n_items), dim3(256), 0, s, items_dev);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// f(theta) and its gradient
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void combine_kernel(const CombineItem *__restrict__ items) {
  const CombineItem ci = items[blockIdx.x];
  const ModelDev &M = *ci.model;
  const int tid = threadIdx.x;
  __shared__ double red[4 * 256];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k = tid; k < kTermBlocks; k += 256) {
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] += ci.term_part[k * 4 + q];
  }
  block_reduce<256>(v, red);
  const double q0 = red[0], q1 = red[256], q2 = red[512], rss = red[768];
  __syncthreads();
  double tp[4] = {0.0, 0.0, 0.0, 0.0}, tc[4] = {0.0, 0.0, 0.0, 0.0};
  const int ntr = (M.nt + 1) * kTraceBlocks;
  if (ci.trp) {
    for (int k = tid; k < ntr; k += 256) {
#pragma unroll
      for (int q = 0; q < 4; ++q) tp[q] += ci.trp[k * 4 + q];
    }
  }
  block_reduce<256>(tp, red);
  double trp[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) trp[q] = red[q * 256];
  __syncthreads();
  if (ci.trc) {
    for (int k = tid; k < ntr; k += 256) {
#pragma unroll
      for (int q = 0; q < 4; ++q) tc[q] += ci.trc[k * 4 + q];
    }
  }
  block_reduce<256>(tc, red);
  double trc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) trc[q] = red[q * 256];
  if (tid != 0) return;
  const double *th = ci.theta;
  const double tauy = exp(th[3]);
  double qb = 0.0;
  const double *muA = ci.mu + (long long)M.nt * M.b;
  for (int k = 0; k < M.a; ++k) qb += muA[k] * muA[k];
  qb *= M.beta_prec;
  double logprior = 0.0;
  for (int k = 0; k < 4; ++k) {
    const double d = th[k] - M.prior_mean[k];
    logprior += 0.5 * log(M.prior_prec[k] / (2.0 * M_PI)) - 0.5 * M.prior_prec[k] * d * d;
  }
  const double mm = (double)M.m;
  const double ldp = ci.logdet[0], ldc = ci.logdet[1];
  // status: 3 = theta outside the parameter space (non-finite, or |rho| = 1 in
  // floating point), 1 / 2 = Q_prior / Q_c not positive definite
  bool bad_theta = false;
  for (int k = 0; k < 4; ++k) bad_theta = bad_theta || !isfinite(th[k]);
  bad_theta = bad_theta || !(fabs(tanh(th[2])) < 1.0);
  const int st = bad_theta ? 3 : (ci.info[0] ? 1 : (ci.info[1] ? 2 : 0));
  double f = -logprior - 0.5 * ldp + 0.5 * (q0 + qb) - 0.5 * mm * th[3] + 0.5 * tauy * rss +
             0.5 * ldc + 0.5 * mm * log(2.0 * M_PI);
  if (st) f = NAN;
  *ci.f = f;
  if (ci.status) *ci.status = st;
  if (ci.grad) {
    const double mean_terms[4] = {2.0 * q0, q1, q2, 0.0};
    for (int k = 0; k < 4; ++k) {
      double g = M.prior_prec[k] * (th[k] - M.prior_mean[k]) - 0.5 * trp[k] + 0.5 * trc[k] +
                 0.5 * mean_terms[k];
      if (k == 3) g += 0.5 * tauy * rss - 0.5 * mm;
      ci.grad[k] = st ? NAN : g;
    }
  }
}

// ---------------------------------------------------------------------------
// two-sided elimination: arrow accumulator and the middle block's hand-over
// ---------------------------------------------------------------------------

__global__ void twist_arrow_kernel(const TwistPair *__restrict__ pairs, int mode) {
  const TwistPair P = pairs[blockIdx.y];
  const int n = P.a * P.a;
  for (int k = blockIdx.x * 256 + threadIdx.x; k < n; k += gridDim.x * 256) {
    if (mode == 0) P.TB[k] = 0.0;
    else P.T[k] += P.TB[k];
  }
}

hipError_t launch_twist_arrow(const TwistPair *pairs_dev, int n_pairs, int max_a, int mode,
                              hipStream_t s) {
  if (n_pairs <= 0 || max_a <= 0) return hipSuccess;
  const int gx = std::min((max_a * max_a + 255) / 256, 16);
  hipLaunchKernelGGL(twist_arrow_kernel, dim3(gx, n_pairs), dim3(256), 0, s, pairs_dev, mode);
  return hipGetLastError();
}

__global__ void twist_middle_kernel(const TwistPair *__restrict__ pairs, int t) {
  const TwistPair P = pairs[blockIdx.y];
  if (P.m != t) return;
  const long long nd = (long long)P.b * P.b, nr = (long long)P.a * P.b;
  for (long long k = blockIdx.x * 256LL + threadIdx.x; k < nd + nr; k += (long long)gridDim.x * 256) {
    if (k < nd) P.SDb[k] = P.SDf[k];
    else P.SRb[k - nd] = P.SRf[k - nd];
  }
}

hipError_t launch_twist_middle(const TwistPair *pairs_dev, int n_pairs, int max_b, int max_a, int t,
                               hipStream_t s) {
  if (n_pairs <= 0) return hipSuccess;
  const long long n = (long long)max_b * max_b + (long long)max_a * max_b;
  const int gx = (int)std::min<long long>((n + 255) / 256, 512);
  hipLaunchKernelGGL(twist_middle_kernel, dim3(gx, n_pairs), dim3(256), 0, s, pairs_dev, t);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// latent marginals over integration points: the mixture of the Gaussians
// N(mu^k, v^k) with weights w_k (the numerical integral of eq. LatParam),
// accumulated chunk by chunk about a shift (the mode's mu) so that the
// variance is not a difference of two large second moments
// ---------------------------------------------------------------------------

__global__ void mixture_accumulate_kernel(const double *__restrict__ mu, const double *__restrict__ var,
                                          const double *__restrict__ w, int K, long long n,
                                          const double *__restrict__ shift, double *acc_m,
                                          double *acc_s, int init) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    double m = init ? 0.0 : acc_m[i], s2 = init ? 0.0 : acc_s[i];
    const double c = shift[i];
    for (int k = 0; k < K; ++k) {
      const double d = mu[(long long)k * n + i] - c;
      m = fma(w[k], d, m);
      s2 = fma(w[k], fma(d, d, var[(long long)k * n + i]), s2);
    }
    acc_m[i] = m;
    acc_s[i] = s2;
  }
}

__global__ void mixture_finish_kernel(const double *__restrict__ shift, const double *__restrict__ acc_m,
                                      const double *__restrict__ acc_s, long long n, double *mean_out,
                                      double *var_out) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    const double m = acc_m[i];
    if (mean_out) mean_out[i] = shift[i] + m;
    if (var_out) var_out[i] = acc_s[i] - m * m;
  }
}

hipError_t launch_mixture_accumulate(const double *mu, const double *var, const double *w, int K,
                                     long long n, const double *shift, double *acc_m, double *acc_s,
                                     int init, hipStream_t s) {
  if (n <= 0 || K <= 0) return hipSuccess;
  const int gx = (int)std::min<long long>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(mixture_accumulate_kernel, dim3(gx), dim3(256), 0, s, mu, var, w, K, n, shift,
                     acc_m, acc_s, init);
  return hipGetLastError();
}

hipError_t launch_mixture_finish(const double *shift, const double *acc_m, const double *acc_s,
                                 long long n, double *mean_out, double *var_out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int gx = (int)std::min<long long>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(mixture_finish_kernel, dim3(gx), dim3(256), 0, s, shift, acc_m, acc_s, n,
                     mean_out, var_out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Poisson likelihood: the pieces of the inner Newton loop and of the implicit
// gradient term (every sum in a fixed order: fixed grids, tree reductions,
// partials summed by the host in block order)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void ng_obs_kernel(const ModelDev *__restrict__ Mp, const double *x,
                                                     double *e_out, double *w_out, double *part) {
  const ModelDev &M = *Mp;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < M.m; i += (long long)gridDim.x * 256) {
    double eta = 0.0;
    for (long long k = M.A_rowptr[i]; k < M.A_rowptr[i + 1]; ++k) eta = fma(M.A_val[k], x[M.A_col[k]], eta);
    const double ex = exp(eta), y = M.y[i];
    if (e_out) e_out[i] = ex;
    if (w_out) w_out[i] = fma(ex, eta - 1.0, y);
    v[0] += y * eta - ex;
  }
  __shared__ double red[4 * 256];
  block_reduce<256>(v, red);
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// The first gsp workgroups take the space-time columns (a few observations
// each) one per lane; each further workgroup takes one fixed-effect column
// (every observation) with a tree over its entries.
__global__ __launch_bounds__(256) void ng_atv_kernel(const ModelDev *__restrict__ Mp, const double *v,
                                                     double *out, int gsp) {
  const ModelDev &M = *Mp;
  const long long nst = (long long)M.b * M.nt;
  if ((int)blockIdx.x < gsp) {
    for (long long j = blockIdx.x * 256LL + threadIdx.x; j < nst; j += (long long)gsp * 256) {
      double acc = 0.0;
      for (long long k = M.Ac_ptr[j]; k < M.Ac_ptr[j + 1]; ++k) acc = fma(M.Ac_val[k], v[M.Ac_row[k]], acc);
      out[j] = acc;
    }
    return;
  }
  const long long j = nst + (blockIdx.x - gsp);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (long long k = M.Ac_ptr[j] + threadIdx.x; k < M.Ac_ptr[j + 1]; k += 256)
    acc[0] = fma(M.Ac_val[k], v[M.Ac_row[k]], acc[0]);
  __shared__ double red[4 * 256];
  block_reduce<256>(acc, red);
  if (threadIdx.x == 0) out[j] = red[0];
}

// D entries: the observations common to the columns of nodes r and s of block
// t (both lists ascending); R rows: the observations of node s times Z.
__global__ void ng_add_obs_kernel(const ModelDev *__restrict__ Mp, const double *e, double *D, double *R) {
  const ModelDev &M = *Mp;
  const int b = M.b, a = M.a, nnz = M.nnz;
  const long long nD = (long long)M.nt * nnz, nR = (long long)M.nt * b * a;
  for (long long idx = blockIdx.x * 256LL + threadIdx.x; idx < nD + nR; idx += (long long)gridDim.x * 256) {
    if (idx < nD) {
      const int t = (int)(idx / nnz), q = (int)(idx % nnz);
      const int r = M.rowidx[q], c = M.colidx[q];
      const long long j1 = (long long)t * b + r, j2 = (long long)t * b + c;
      long long p1 = M.Ac_ptr[j1], p2 = M.Ac_ptr[j2];
      const long long q1 = M.Ac_ptr[j1 + 1], q2 = M.Ac_ptr[j2 + 1];
      double acc = 0.0;
      while (p1 < q1 && p2 < q2) {
        const int i1 = M.Ac_row[p1], i2 = M.Ac_row[p2];
        if (i1 == i2) {
          acc = fma(e[i1] * M.Ac_val[p1], M.Ac_val[p2], acc);
          ++p1;
          ++p2;
        } else if (i1 < i2) {
          ++p1;
        } else {
          ++p2;
        }
      }
      D[(long long)t * b * b + r + (long long)c * b] += acc;
    } else {
      const long long q = idx - nD;
      const int t = (int)(q / ((long long)b * a));
      const int rem = (int)(q - (long long)t * b * a);
      const int c = rem / a, al = rem % a;
      const long long j = (long long)t * b + c;
      double acc = 0.0;
      for (long long k = M.Ac_ptr[j]; k < M.Ac_ptr[j + 1]; ++k) {
        const int i = M.Ac_row[k];
        acc = fma(e[i] * M.Ac_val[k], M.Zd[(long long)i * a + al], acc);
      }
      R[(long long)t * a * b + al + (long long)c * a] += acc;
    }
  }
}

// T += Z^T diag(e) Z: one workgroup per entry, a tree over the observations.
__global__ __launch_bounds__(256) void ng_add_T_kernel(const ModelDev *__restrict__ Mp, const double *e,
                                                       double *T) {
  const ModelDev &M = *Mp;
  const int a = M.a, al = blockIdx.x % a, be = blockIdx.x / a;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (long long i = threadIdx.x; i < M.m; i += 256)
    v[0] = fma(e[i] * M.Zd[i * a + al], M.Zd[i * a + be], v[0]);
  __shared__ double red[4 * 256];
  block_reduce<256>(v, red);
  if (threadIdx.x == 0) T[al + (long long)be * a] += red[0];
}

__global__ void ng_obs_var_kernel(const ModelDev *__restrict__ Mp, const double *SD, const double *SR,
                                  const double *ST, const double *e, double *c_out) {
  const ModelDev &M = *Mp;
  const int b = M.b, a = M.a;
  const long long nst = (long long)b * M.nt;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < M.m; i += (long long)gridDim.x * 256) {
    const long long k0 = M.A_rowptr[i], k1 = M.A_rowptr[i + 1];
    double q = 0.0;
    for (long long k = k0; k < k1; ++k) {
      const long long ck = M.A_col[k];
      const double ak = M.A_val[k];
      if (ck < nst) {
        const long long t = ck / b;
        const int r = (int)(ck - t * b);
        for (long long l = k0; l < k1; ++l) {
          const long long cl = M.A_col[l];
          if (cl < nst) {
            const int c = (int)(cl - t * b);   // same time block (checked at model creation)
            q = fma(ak * M.A_val[l], SD[t * b * b + r + (long long)c * b], q);
          } else {
            const int al = (int)(cl - nst);
            q = fma(2.0 * ak * M.A_val[l], SR[t * a * b + al + (long long)r * a], q);
          }
        }
      } else {
        const int al = (int)(ck - nst);
        for (long long l = k0; l < k1; ++l) {
          const long long cl = M.A_col[l];
          if (cl >= nst) q = fma(ak * M.A_val[l], ST[al + (cl - nst) * a], q);
        }
      }
    }
    c_out[i] = 0.5 * e[i] * q;
  }
}

__global__ __launch_bounds__(256) void ng_quad_kernel(const ModelDev *__restrict__ Mp, const double *theta,
                                                      const double *u, const double *v, double *part) {
  const ModelDev &M = *Mp;
  const int b = M.b, nt = M.nt;
  const Coef c = make_coef(M, theta);
  const double cS = ar1_off(c), dcS = ar1_doff(c);
  const long long nst = (long long)nt * b;
  const long long stride = (long long)gridDim.x * blockDim.x;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < nst; idx += stride) {
    const int t = (int)(idx / b), s = (int)(idx % b);
    const bool nx = t < nt - 1;
    const double *ut1 = u + (long long)(t + 1) * b, *vt = v + (long long)t * b, *vt1 = vt + b;
    double qv0 = 0.0, dv0 = 0.0, qv1 = 0.0, dv1 = 0.0, qu1 = 0.0, du1 = 0.0;
    for (int e = M.colptr[s]; e < M.colptr[s + 1]; ++e) {
      const int i = M.rowidx[e];
      const double q = qs_entry(M, c, e), dq = dqs_entry(M, c, e);
      qv0 += q * vt[i];
      dv0 += dq * vt[i];
      if (nx) {
        qv1 += q * vt1[i];
        dv1 += dq * vt1[i];
        qu1 += q * ut1[i];
        du1 += dq * ut1[i];
      }
    }
    const double us = u[idx], vs = v[idx];
    const double cD = ar1_diag(c, t, nt), dcD = ar1_ddiag(c, t, nt);
    // u_t^T Q_s v_t cD + (u_t^T Q_s v_{t+1} + u_{t+1}^T Q_s v_t) cS, term by term
    acc[0] += us * (cD * qv0 + cS * qv1) + vs * cS * qu1;
    acc[1] += us * (cD * dv0 + cS * dv1) + vs * cS * du1;
    acc[2] += us * (dcD * qv0 + dcS * qv1) + vs * dcS * qu1;
  }
  for (long long j = nst + blockIdx.x * (long long)blockDim.x + threadIdx.x; j < M.n; j += stride)
    acc[3] += u[j] * v[j];
  __shared__ double red[4 * 256];
  block_reduce<256>(acc, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) part[(long long)blockIdx.x * 4 + k] = red[k * 256];
  }
}

__global__ __launch_bounds__(256) void ng_step_kernel(const double *x, const double *xn, double step,
                                                      double *cand, long long n, double *part) {
  double dmax = 0.0, xmax = 0.0;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    const double xi = x[i];
    const double ci = fma(step, xn[i] - xi, xi);
    cand[i] = ci;
    dmax = fmax(dmax, fabs(ci - xi));
    xmax = fmax(xmax, fabs(xi));
  }
  __shared__ double r0[256], r1[256];
  r0[threadIdx.x] = dmax;
  r1[threadIdx.x] = xmax;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      r0[threadIdx.x] = fmax(r0[threadIdx.x], r0[threadIdx.x + off]);
      r1[threadIdx.x] = fmax(r1[threadIdx.x], r1[threadIdx.x + off]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x * 2] = r0[0];
    part[blockIdx.x * 2 + 1] = r1[0];
  }
}

hipError_t launch_ng_obs(const ModelDev *M, long long m, const double *x, double *e_out, double *w_out,
                         double *part, hipStream_t s) {
  (void)m;
  hipLaunchKernelGGL(ng_obs_kernel, dim3(kNgBlocks), dim3(256), 0, s, M, x, e_out, w_out, part);
  return hipGetLastError();
}
hipError_t launch_ng_atv(const ModelDev *M, long long nst, int a, const double *v, double *out,
                         hipStream_t s) {
  const int gsp = (int)std::max<long long>(1, std::min<long long>((nst + 255) / 256, 4096));
  hipLaunchKernelGGL(ng_atv_kernel, dim3(gsp + a), dim3(256), 0, s, M, v, out, gsp);
  return hipGetLastError();
}
hipError_t launch_ng_add_obs(const ModelDev *M, int b, int nt, int a, int nnz, const double *e, double *D,
                             double *R, double *T, hipStream_t s) {
  const long long tot = (long long)nt * nnz + (long long)nt * b * a;
  const int gx = (int)std::max<long long>(1, std::min<long long>((tot + 255) / 256, 8192));
  hipLaunchKernelGGL(ng_add_obs_kernel, dim3(gx), dim3(256), 0, s, M, e, D, R);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess || a == 0) return err;
  hipLaunchKernelGGL(ng_add_T_kernel, dim3(a * a), dim3(256), 0, s, M, e, T);
  return hipGetLastError();
}
hipError_t launch_ng_obs_var(const ModelDev *M, long long m, const double *SD, const double *SR,
                             const double *ST, const double *e, double *c_out, hipStream_t s) {
  const int gx = (int)std::max<long long>(1, std::min<long long>((m + 255) / 256, 4096));
  hipLaunchKernelGGL(ng_obs_var_kernel, dim3(gx), dim3(256), 0, s, M, SD, SR, ST, e, c_out);
  return hipGetLastError();
}
hipError_t launch_ng_quad(const ModelDev *M, const double *theta, const double *u, const double *v,
                          double *part, hipStream_t s) {
  hipLaunchKernelGGL(ng_quad_kernel, dim3(kNgBlocks), dim3(256), 0, s, M, theta, u, v, part);
  return hipGetLastError();
}
hipError_t launch_ng_step(const double *x, const double *xn, double step, double *cand, long long n,
                          double *part, hipStream_t s) {
  hipLaunchKernelGGL(ng_step_kernel, dim3(kNgBlocks), dim3(256), 0, s, x, xn, step, cand, n, part);
  return hipGetLastError();
}

hipError_t launch_combine(const CombineItem *items_dev, int n_items, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(combine_kernel, dim3(n_items), dim3(256), 0, s, items_dev);
  return hipGetLastError();
}

}  // namespace inla
