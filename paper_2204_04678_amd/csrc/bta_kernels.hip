// Block kernels of the BTA Cholesky factorization and selected inversion.
//
// Every kernel launch covers one phase of one time step for a whole batch of
// BTA matrices ("items").  Workgroup g of the launch finds its item by walking
// the items' task counts (phase_tasks), decodes its task (an output tile plus
// up to three products A B^T summed into it), and runs it on the FP64 matrix
// cores (v_mfma_f64_16x16x4f64).  Paper: Sec. "Sparse Linear Algebra" for the
// factorization and log-determinant, Sec. "Partial Inversion" for the
// selected inversion; the block recursions are written out in the host engine.
#include <climits>

#include "inla_internal.h"

namespace inla {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int KC = 16;            // k-chunk staged through LDS
constexpr int LDP = kTile + 2;    // LDS row length of a [k][row] operand panel
constexpr int TLD = kTile + 1;    // LDS row length of a full 64 x 64 tile
constexpr int kLeanLds = 2 * KC * LDP;
constexpr int kFatLds = 2 * kTile * TLD + kTile + 64;

struct Seg {
  const double *A;
  long long ars, aks;             // op(A)(r, k) = A[r*ars + k*aks]
  const double *B;
  long long brs, bks;             // op(B)(c, k) = B[c*brs + k*bks];  product = op(A) op(B)^T
  int k0, k1;
  double alpha;
};

enum TaskKind { TK_NONE = 0, TK_PRODUCT = 1, TK_COPY = 2, TK_ZERO = 3 };

struct Task {
  int kind;
  int m, n;                       // output tile rows, cols
  double *C;
  long long ldc;
  double beta;                    // C = beta*C + sum_s alpha_s op(A_s) op(B_s)^T
  int nseg;
  Seg seg[3];
  int mirror;                     // also store C^T at Cm (symmetric output)
  int diagtile;                   // mirror: lower entries only
  double *Cm;
  int chol;                       // Cholesky + inverse of the result tile -> Lout
  double *Lout;
  long long ldl;
  double *ldsum;
  int row_off;
  int left;                       // C = -E P with E a lower-triangular tile
  const double *E;
  long long lde;
  const double *src;              // copy source (ld = ldc)
};

__device__ inline int tdim(int n, int i) { return min(kTile, n - i * kTile); }
__device__ inline long long toff(int b, int i, int j) {
  return (long long)i * kTile + (long long)j * kTile * b;
}
__device__ inline void tri_decode(int q, int &i, int &j) {
  int r = (int)((sqrt(8.0 * q + 1.0) - 1.0) * 0.5);
  while ((r + 1) * (r + 2) / 2 <= q) ++r;
  while (r * (r + 1) / 2 > q) --r;
  i = r;
  j = q - r * (r + 1) / 2;
}
__device__ inline void set_seg(Seg &g, const double *A, long long ars, long long aks, const double *B,
                               long long brs, long long bks, int k0, int k1, double alpha) {
  g.A = A; g.ars = ars; g.aks = aks; g.B = B; g.brs = brs; g.bks = bks;
  g.k0 = k0; g.k1 = k1; g.alpha = alpha;
}

// Map (item, phase, t, p, local task q) to the work of one workgroup.
__device__ void decode(const ItemDev &it, int phase, int t, int p, int q, Task &tk) {
  const int b = it.b, a = it.a, nP = it.nP;
  const long long bb = (long long)b * b;
  const bool arrow = a > 0;
  const bool last = (t == it.nt - 1);
  tk.kind = TK_PRODUCT; tk.nseg = 0; tk.beta = 0.0; tk.mirror = 0; tk.diagtile = 0; tk.chol = 0;
  tk.left = 0; tk.Cm = nullptr; tk.Lout = nullptr; tk.ldsum = nullptr; tk.E = nullptr;
  tk.src = nullptr; tk.ldl = 0; tk.lde = 0; tk.row_off = 0;
  double *Dt = it.D + (long long)t * bb;
  double *St = it.S ? it.S + (long long)t * bb : nullptr;
  double *Rt = arrow ? it.R + (long long)t * a * b : nullptr;
  switch (phase) {
    case PH_DIAG0: {
      tk.m = tk.n = tdim(b, 0);
      tk.C = Dt; tk.ldc = b; tk.beta = 1.0;
      tk.chol = 1; tk.Lout = it.W1; tk.ldl = b;
      tk.ldsum = it.ldpart + (long long)t * nP; tk.row_off = t * b;
      return;
    }
    case PH_PANEL: {
      if (q < nP - 1 - p) {
        const int i = p + 1 + q;
        tk.m = tdim(b, i); tk.n = tdim(b, p);
        tk.C = Dt + toff(b, i, p); tk.ldc = b;
        set_seg(tk.seg[0], Dt + toff(b, i, p), 1, b, it.W1 + toff(b, p, p), 1, b, 0, tdim(b, p), 1.0);
        tk.nseg = 1;
      } else {
        const int j = q - (nP - 1 - p);
        tk.m = tdim(b, p); tk.n = tdim(b, j);
        tk.C = it.W1 + toff(b, p, j); tk.ldc = b;
        set_seg(tk.seg[0], Dt + (long long)p * kTile, 1, b, it.W1 + (long long)j * kTile * b, b, 1,
                j * kTile, p * kTile, 1.0);
        tk.nseg = 1;
        tk.left = 1; tk.E = it.W1 + toff(b, p, p); tk.lde = b;
      }
      return;
    }
    case PH_TRAIL: {
      const int n2 = nP - 1 - p;
      const int cnt = n2 * (n2 + 1) / 2;
      if (q < cnt) {
        int ii, jj;
        tri_decode(q, ii, jj);
        const int i = p + 1 + ii, j = p + 1 + jj;
        tk.m = tdim(b, i); tk.n = tdim(b, j);
        tk.C = Dt + toff(b, i, j); tk.ldc = b; tk.beta = 1.0;
        set_seg(tk.seg[0], Dt + toff(b, i, p), 1, b, Dt + toff(b, j, p), 1, b, 0, tdim(b, p), -1.0);
        tk.nseg = 1;
        if (i == p + 1 && j == p + 1) {
          tk.chol = 1; tk.Lout = it.W1 + toff(b, i, i); tk.ldl = b;
          tk.ldsum = it.ldpart + (long long)t * nP + i; tk.row_off = t * b + i * kTile;
        }
      } else {
        const int j = q - cnt;
        tk.kind = TK_COPY;
        tk.m = tdim(b, p); tk.n = tdim(b, j);
        tk.src = it.W1 + toff(b, p, j); tk.C = Dt + toff(b, p, j); tk.ldc = b;
      }
      return;
    }
    case PH_OFFDIAG: {
      int idx = q;
      if (!last) {
        if (idx < nP * nP) {
          const int i = idx / nP, j = idx % nP;
          tk.m = tdim(b, i); tk.n = tdim(b, j);
          tk.C = it.W2 + toff(b, i, j); tk.ldc = b;
          set_seg(tk.seg[0], St + (long long)i * kTile, 1, b, it.W1 + (long long)j * kTile, 1, b, 0,
                  min(b, (j + 1) * kTile), 1.0);
          tk.nseg = 1;
          return;
        }
        idx -= nP * nP;
      }
      if (arrow) {
        if (idx < nP) {
          const int j = idx;
          tk.m = a; tk.n = tdim(b, j);
          tk.C = it.W3 + (long long)j * kTile * a; tk.ldc = a;
          set_seg(tk.seg[0], Rt, 1, a, it.W1 + (long long)j * kTile, 1, b, 0, min(b, (j + 1) * kTile),
                  1.0);
          tk.nseg = 1;
          return;
        }
        idx -= nP;
      }
      if (idx < nP) {
        const int j = idx;
        tk.kind = TK_COPY;
        tk.m = tdim(b, nP - 1); tk.n = tdim(b, j);
        tk.src = it.W1 + toff(b, nP - 1, j); tk.C = Dt + toff(b, nP - 1, j); tk.ldc = b;
        return;
      }
      idx -= nP;
      {
        // strictly upper tile (i, j), j > i, of the factor block: stored as zeros
        int jj, ii;
        tri_decode(idx, jj, ii);   // jj > ii enumerates pairs with j in 1..nP-1, i < j
        const int j = jj + 1, i = ii;
        tk.kind = TK_ZERO;
        tk.m = tdim(b, i); tk.n = tdim(b, j);
        tk.C = Dt + toff(b, i, j); tk.ldc = b;
      }
      return;
    }
    case PH_SCHUR: {
      int idx = q;
      if (!last) {
        const int c1 = nP * (nP + 1) / 2;
        if (idx < c1) {
          int i, j;
          tri_decode(idx, i, j);
          tk.m = tdim(b, i); tk.n = tdim(b, j);
          tk.C = it.D + (long long)(t + 1) * bb + toff(b, i, j); tk.ldc = b; tk.beta = 1.0;
          set_seg(tk.seg[0], it.W2 + (long long)i * kTile, 1, b, it.W2 + (long long)j * kTile, 1, b, 0,
                  b, -1.0);
          tk.nseg = 1;
          return;
        }
        idx -= c1;
        if (idx < nP * nP) {
          const int i = idx / nP, j = idx % nP;
          tk.kind = TK_COPY;
          tk.m = tdim(b, i); tk.n = tdim(b, j);
          tk.src = it.W2 + toff(b, i, j); tk.C = St + toff(b, i, j); tk.ldc = b;
          return;
        }
        idx -= nP * nP;
      }
      if (arrow) {
        if (!last) {
          if (idx < nP) {
            const int j = idx;
            tk.m = a; tk.n = tdim(b, j);
            tk.C = it.R + (long long)(t + 1) * a * b + (long long)j * kTile * a; tk.ldc = a;
            tk.beta = 1.0;
            set_seg(tk.seg[0], it.W3, 1, a, it.W2 + (long long)j * kTile, 1, b, 0, b, -1.0);
            tk.nseg = 1;
            return;
          }
          idx -= nP;
        }
        if (idx == 0) {
          tk.m = a; tk.n = a;
          tk.C = it.T; tk.ldc = a; tk.beta = 1.0;
          set_seg(tk.seg[0], it.W3, 1, a, it.W3, 1, a, 0, b, -1.0);
          tk.nseg = 1;
          return;
        }
        idx -= 1;
        const int j = idx;
        tk.kind = TK_COPY;
        tk.m = a; tk.n = tdim(b, j);
        tk.src = it.W3 + (long long)j * kTile * a; tk.C = Rt + (long long)j * kTile * a; tk.ldc = a;
        return;
      }
      tk.kind = TK_NONE;
      return;
    }
    case PH_ARROW: {
      tk.m = tk.n = a;
      tk.C = it.T; tk.ldc = a; tk.beta = 1.0;
      tk.chol = 1; tk.Lout = it.T; tk.ldl = a;
      tk.ldsum = it.ldpart + (long long)it.nt * nP; tk.row_off = it.nt * b;
      return;
    }
    case PH_SI_INIT: {
      tk.m = tk.n = a;
      tk.C = it.ST; tk.ldc = a;
      set_seg(tk.seg[0], it.T, a, 1, it.T, a, 1, 0, a, 1.0);
      tk.nseg = 1;
      return;
    }
    case PH_SI_VU: {
      int idx = q;
      if (!last) {
        if (idx < nP * nP) {
          const int i = idx / nP, j = idx % nP;
          tk.m = tdim(b, i); tk.n = tdim(b, j);
          tk.C = it.W2 + toff(b, i, j); tk.ldc = b;
          set_seg(tk.seg[0], St + (long long)i * kTile, 1, b, Dt + (long long)j * kTile * b, b, 1,
                  j * kTile, b, 1.0);
          tk.nseg = 1;
          return;
        }
        idx -= nP * nP;
      }
      const int j = idx;
      tk.m = a; tk.n = tdim(b, j);
      tk.C = it.W3 + (long long)j * kTile * a; tk.ldc = a;
      set_seg(tk.seg[0], Rt, 1, a, Dt + (long long)j * kTile * b, b, 1, j * kTile, b, 1.0);
      tk.nseg = 1;
      return;
    }
    case PH_SI_SR: {
      int idx = q;
      double *SDn = last ? nullptr : sig_D(it, t + 1);
      double *SRn = (last || !arrow) ? nullptr : sig_R(it, t + 1);
      if (!last) {
        if (idx < nP * nP) {
          const int i = idx / nP, j = idx % nP;
          tk.m = tdim(b, i); tk.n = tdim(b, j);
          tk.C = sig_S(it, t) + toff(b, i, j); tk.ldc = b;
          set_seg(tk.seg[0], SDn + (long long)i * kTile, 1, b, it.W2 + (long long)j * kTile * b, b, 1,
                  0, b, -1.0);
          tk.nseg = 1;
          if (arrow) {
            set_seg(tk.seg[1], SRn + (long long)i * kTile * a, a, 1, it.W3 + (long long)j * kTile * a,
                    a, 1, 0, a, -1.0);
            tk.nseg = 2;
          }
          return;
        }
        idx -= nP * nP;
      }
      const int j = idx;
      tk.m = a; tk.n = tdim(b, j);
      tk.C = sig_R(it, t) + (long long)j * kTile * a; tk.ldc = a;
      if (!last) {
        set_seg(tk.seg[0], SRn, 1, a, it.W2 + (long long)j * kTile * b, b, 1, 0, b, -1.0);
        set_seg(tk.seg[1], it.ST, 1, a, it.W3 + (long long)j * kTile * a, a, 1, 0, a, -1.0);
        tk.nseg = 2;
      } else {
        set_seg(tk.seg[0], it.ST, 1, a, it.W3 + (long long)j * kTile * a, a, 1, 0, a, -1.0);
        tk.nseg = 1;
      }
      return;
    }
    case PH_SI_SD: {
      int i, j;
      tri_decode(q, i, j);
      double *SDt = sig_D(it, t);
      tk.m = tdim(b, i); tk.n = tdim(b, j);
      tk.C = SDt + toff(b, i, j); tk.ldc = b;
      tk.mirror = 1; tk.Cm = SDt + toff(b, j, i); tk.diagtile = (i == j);
      set_seg(tk.seg[0], Dt + (long long)i * kTile * b, b, 1, Dt + (long long)j * kTile * b, b, 1,
              i * kTile, b, 1.0);
      tk.nseg = 1;
      if (!last) {
        set_seg(tk.seg[1], sig_S(it, t) + (long long)i * kTile * b, b, 1,
                it.W2 + (long long)j * kTile * b, b, 1, 0, b, -1.0);
        tk.nseg = 2;
        if (arrow) {
          set_seg(tk.seg[2], sig_R(it, t) + (long long)i * kTile * a, a, 1,
                  it.W3 + (long long)j * kTile * a, a, 1, 0, a, -1.0);
          tk.nseg = 3;
        }
      } else if (arrow) {
        set_seg(tk.seg[1], sig_R(it, t) + (long long)i * kTile * a, a, 1,
                it.W3 + (long long)j * kTile * a, a, 1, 0, a, -1.0);
        tk.nseg = 2;
      }
      return;
    }
    default:
      tk.kind = TK_NONE;
      return;
  }
}

// Stage rows [0, rows) x k in [kc, min(kc+KC, k1)) of op(X) into P[k][row] (zero-filled).
__device__ inline void load_panel(double *P, const double *X, long long rs, long long ks, int rows,
                                  int kc, int k1, double alpha) {
  const int tid = threadIdx.x;
  if (rs == 1) {
#pragma unroll
    for (int q = 0; q < (KC * kTile) / kThreads; ++q) {
      const int e = tid + q * kThreads;
      const int r = e & (kTile - 1), k = e / kTile;
      const int kk = kc + k;
      double v = 0.0;
      if (r < rows && kk < k1) v = alpha * X[(long long)r + (long long)kk * ks];
      P[k * LDP + r] = v;
    }
  } else {
#pragma unroll
    for (int q = 0; q < (KC * kTile) / kThreads; ++q) {
      const int e = tid + q * kThreads;
      const int k = e & (KC - 1), r = e / KC;
      const int kk = kc + k;
      double v = 0.0;
      if (r < rows && kk < k1) v = alpha * X[(long long)r * rs + (long long)kk * ks];
      P[k * LDP + r] = v;
    }
  }
}

// acc += op(A) op(B)^T over all segments of the task.
__device__ void run_product(const Task &tk, double *smem, d4 (&acc)[2][2]) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w >> 1, wc = w & 1;
  double *As = smem;
  double *Bs = smem + KC * LDP;
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    if (s >= tk.nseg) break;
    const Seg g = tk.seg[s];
    for (int kc = g.k0; kc < g.k1; kc += KC) {
      load_panel(As, g.A, g.ars, g.aks, tk.m, kc, g.k1, g.alpha);
      load_panel(Bs, g.B, g.brs, g.bks, tk.n, kc, g.k1, 1.0);
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < KC; kk += 4) {
        const int kr = (kk + (lane >> 4)) * LDP;
        const double a0 = As[kr + wr * 32 + (lane & 15)];
        const double a1 = As[kr + wr * 32 + 16 + (lane & 15)];
        const double b0 = Bs[kr + wc * 32 + (lane & 15)];
        const double b1 = Bs[kr + wc * 32 + 16 + (lane & 15)];
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
      }
      __syncthreads();
    }
  }
}

// Output mapping of v_mfma_f64_16x16x4f64: lane l, element r -> row (l>>4) + 4r, col l&15.
__device__ inline int acc_row(int wr, int mi, int lane, int r) {
  return wr * 32 + mi * 16 + (lane >> 4) + 4 * r;
}
__device__ inline int acc_col(int wc, int nj, int lane) { return wc * 32 + nj * 16 + (lane & 15); }

// Cholesky of the lower triangle of the w x w tile A (LDS, row-major, ld TLD)
// followed by the inverse of the factor.  Columns are kept unscaled during the
// elimination (A_j[i][k] -= A_j[i][j] A_j[k][j] / A_j[j][j]), so one barrier
// per column suffices; then V = unit-lower factor, Y = V^{-1} by forward
// substitution, and inv(L) = diag(1/l) Y with l_j = sqrt(pivot_j).
__device__ void chol_inv_tile(double *A, double *X, double *dl, int w, double *Lout, long long ldl,
                              double *ldsum, int row_off, int *info) {
  const int tid = threadIdx.x;
  const int ntri = w * (w + 1) / 2;
  int ei[9], ek[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const int e = tid + q * kThreads;
    if (e < ntri) {
      int i, k;
      tri_decode(e, i, k);
      ei[q] = i; ek[q] = k;
    } else {
      ei[q] = -1; ek[q] = 0;
    }
  }
  for (int j = 0; j < w; ++j) {
    const double piv = A[j * TLD + j];
    if (tid == 0 && !(piv > 0.0)) atomicMin(info, row_off + j + 1);
    const double inv = 1.0 / piv;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      if (ek[q] > j) A[ei[q] * TLD + ek[q]] -= A[ei[q] * TLD + j] * A[ek[q] * TLD + j] * inv;
    }
    __syncthreads();
  }
  // unit-lower V (in place below the diagonal) and Y = I
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    if (ei[q] >= 0) {
      if (ei[q] > ek[q]) A[ei[q] * TLD + ek[q]] /= A[ek[q] * TLD + ek[q]];
      X[ei[q] * TLD + ek[q]] = (ei[q] == ek[q]) ? 1.0 : 0.0;
    }
  }
  if (tid < w) dl[tid] = sqrt(A[tid * TLD + tid]);
  __syncthreads();
  for (int k = 0; k + 1 < w; ++k) {
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      if (ei[q] > k && ek[q] <= k) X[ei[q] * TLD + ek[q]] -= A[ei[q] * TLD + k] * X[k * TLD + ek[q]];
    }
    __syncthreads();
  }
  // inv(L) = diag(1/l) Y, stored as a full tile with zeros above the diagonal
  for (int e = tid; e < kTile * kTile; e += kThreads) {
    const int r = e & (kTile - 1), c = e / kTile;
    if (r < w && c < w) Lout[r + (long long)c * ldl] = (c <= r) ? X[r * TLD + c] / dl[r] : 0.0;
  }
  if (tid < 64) {
    double v = (tid < w) ? log(dl[tid]) : 0.0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (tid == 0) *ldsum = v;
  }
}

template <bool FAT>
__global__ __launch_bounds__(kThreads) void tile_phase_kernel(const ItemDev *__restrict__ items,
                                                              int n_items, int phase, int t, int p) {
  __shared__ double smem[FAT ? kFatLds : kLeanLds];
  int q = blockIdx.x;
  int ii = 0;
  for (; ii < n_items; ++ii) {
    const int c = phase_tasks(items[ii], phase, t, p);
    if (q < c) break;
    q -= c;
  }
  if (ii >= n_items) return;
  const ItemDev it = items[ii];
  Task tk;
  decode(it, phase, t, p, q, tk);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w >> 1, wc = w & 1;
  if (tk.kind == TK_NONE) return;
  if (tk.kind == TK_COPY || tk.kind == TK_ZERO) {
    for (int e = tid; e < kTile * kTile; e += kThreads) {
      const int r = e & (kTile - 1), c = e / kTile;
      if (r < tk.m && c < tk.n)
        tk.C[r + c * tk.ldc] = (tk.kind == TK_COPY) ? tk.src[r + c * tk.ldc] : 0.0;
    }
    return;
  }
  d4 acc[2][2];
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int nj = 0; nj < 2; ++nj) acc[mi][nj] = d4{0.0, 0.0, 0.0, 0.0};
  run_product(tk, smem, acc);

  if constexpr (FAT) {
    if (tk.chol) {
      double *A = smem;
      double *X = smem + kTile * TLD;
      double *dl = smem + 2 * kTile * TLD;
      for (int e = tid; e < kTile * kTile; e += kThreads) A[(e / kTile) * TLD + (e % kTile)] = 0.0;
      __syncthreads();
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < 2; ++nj)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = acc_row(wr, mi, lane, r), col = acc_col(wc, nj, lane);
            if (row < tk.m && col < tk.n) {
              double v = acc[mi][nj][r];
              if (tk.beta != 0.0) v += tk.beta * tk.C[row + col * tk.ldc];
              A[row * TLD + col] = v;
            }
          }
      __syncthreads();
      chol_inv_tile(A, X, dl, tk.m, tk.Lout, tk.ldl, tk.ldsum, tk.row_off, it.info);
      return;
    }
    if (tk.left) {
      // P (m x n) -> LDS as [k = row of P][col]; E (m x m lower) -> LDS as [k][row]
      double *Pl = smem;
      double *El = smem + kTile * TLD;
      for (int e = tid; e < kTile * kTile; e += kThreads) {
        const int r = e & (kTile - 1), c = e / kTile;
        Pl[c * TLD + r] = 0.0;
        El[c * TLD + r] = (r < tk.m && c < tk.m) ? tk.E[r + c * tk.lde] : 0.0;  // El[k=c][row=r]
      }
      __syncthreads();
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < 2; ++nj)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = acc_row(wr, mi, lane, r), col = acc_col(wc, nj, lane);
            if (row < tk.m && col < tk.n) Pl[row * TLD + col] = acc[mi][nj][r];
          }
      __syncthreads();
      d4 out[2][2];
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < 2; ++nj) out[mi][nj] = d4{0.0, 0.0, 0.0, 0.0};
      for (int kk = 0; kk < kTile; kk += 4) {
        const int k = kk + (lane >> 4);
        const double a0 = El[k * TLD + wr * 32 + (lane & 15)];
        const double a1 = El[k * TLD + wr * 32 + 16 + (lane & 15)];
        const double b0 = Pl[k * TLD + wc * 32 + (lane & 15)];
        const double b1 = Pl[k * TLD + wc * 32 + 16 + (lane & 15)];
        out[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, out[0][0], 0, 0, 0);
        out[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, out[0][1], 0, 0, 0);
        out[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, out[1][0], 0, 0, 0);
        out[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, out[1][1], 0, 0, 0);
      }
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < 2; ++nj)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = acc_row(wr, mi, lane, r), col = acc_col(wc, nj, lane);
            if (row < tk.m && col < tk.n) tk.C[row + col * tk.ldc] = -out[mi][nj][r];
          }
      return;
    }
  }
  // plain (and mirrored) store
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int nj = 0; nj < 2; ++nj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = acc_row(wr, mi, lane, r), col = acc_col(wc, nj, lane);
        if (row < tk.m && col < tk.n) {
          double v = acc[mi][nj][r];
          double *cp = tk.C + row + col * tk.ldc;
          if (tk.beta != 0.0) v += tk.beta * (*cp);
          if (tk.mirror && tk.diagtile) {
            if (row >= col) {
              *cp = v;
              tk.Cm[col + row * tk.ldc] = v;
            }
          } else {
            *cp = v;
            if (tk.mirror) tk.Cm[col + row * tk.ldc] = v;
          }
        }
      }
}

hipError_t launch_tile_phase(const ItemDev *items_dev, int n_items, int total, int phase, int t,
                             int p, hipStream_t s) {
  if (total <= 0) return hipSuccess;
  if (phase_is_fat(phase)) {
    hipLaunchKernelGGL(tile_phase_kernel<true>, dim3(total), dim3(kThreads), 0, s, items_dev, n_items,
                       phase, t, p);
  } else {
    hipLaunchKernelGGL(tile_phase_kernel<false>, dim3(total), dim3(kThreads), 0, s, items_dev,
                       n_items, phase, t, p);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// small utility kernels
// ---------------------------------------------------------------------------

__global__ void fill_kernel(double *p, long long n, double v) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void fill_int_kernel(int *p, long long n, int v) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t launch_fill(double *ptr, long long n, double v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const long long blocks = std::min<long long>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, s, ptr, n, v);
  return hipGetLastError();
}
hipError_t launch_fill_int(int *ptr, long long n, int v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const long long blocks = std::min<long long>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(fill_int_kernel, dim3((unsigned)blocks), dim3(256), 0, s, ptr, n, v);
  return hipGetLastError();
}

// log|Q| = 2 sum of the per-tile partial sums of log L_jj, in a fixed tree order.
__global__ void logdet_finish_kernel(const ItemDev *items, double *logdet_out, int *info_out) {
  const ItemDev it = items[blockIdx.x];
  const int cnt = it.nt * it.nP + (it.a > 0 ? 1 : 0);
  __shared__ double red[256];
  double v = 0.0;
  for (int i = threadIdx.x; i < cnt; i += 256) v += it.ldpart[i];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int inf = *it.info;
    if (info_out) info_out[blockIdx.x] = (inf == kInfoNone) ? 0 : inf;
    if (logdet_out) logdet_out[blockIdx.x] = (inf == kInfoNone) ? 2.0 * red[0] : NAN;
  }
}

hipError_t launch_logdet_finish(const ItemDev *items_dev, int n_items, double *logdet_out,
                                int *info_out, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(logdet_finish_kernel, dim3(n_items), dim3(256), 0, s, items_dev, logdet_out,
                     info_out);
  return hipGetLastError();
}

}  // namespace inla
