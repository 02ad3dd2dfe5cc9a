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
#include <type_traits>

#include "inla_internal.h"

namespace inla {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int LDP = kTile + 2;    // LDS row length of a [k][row] operand panel
constexpr int TLD = kTile + 1;    // LDS row length of a full 64 x 64 tile
constexpr int kLeanKC = 32;       // k-chunk of the product kernel
constexpr int kFatKC = 32;        // k-chunk of the Cholesky-capable kernel
constexpr int kLeanLds = 2 * 2 * kLeanKC * LDP;                      // double-buffered panels
constexpr int kFatLds = 2 * kTile * TLD + 2 * kTile;                 // tile + inverse + logs
static_assert(kFatLds >= 2 * 2 * kFatKC * LDP, "fat LDS must hold the product panels too");
// Product kernel layouts: WR x WC waves over a TS x TS output tile, k-chunk
// KC, register prefetch depth DEPTH (register-staged layouts) or direct loads
// into LDS (DMA), and the minimum waves per SIMD it is built for (OCC).
template <int V> struct BigCfg;
template <> struct BigCfg<0> {   // 128: 8 waves of 64 x 32, two register sets
  static constexpr int TS = 128, WR = 2, WC = 4, KC = 16, DEPTH = 2, OCC = 1;
  static constexpr bool DMA = false;
  static constexpr int STAGES = 2;
};
template <> struct BigCfg<1> {   // 128: 4 waves of 64 x 64, one wave per SIMD
  static constexpr int TS = 128, WR = 2, WC = 2, KC = 16, DEPTH = 2, OCC = 1;
  static constexpr bool DMA = false;
  static constexpr int STAGES = 2;
};
template <> struct BigCfg<2> {   // 128: 8 waves of 64 x 32, deeper k-chunk, one register set
  static constexpr int TS = 128, WR = 2, WC = 4, KC = 32, DEPTH = 1, OCC = 1;
  static constexpr bool DMA = false;
  static constexpr int STAGES = 2;
};
template <> struct BigCfg<3> {   // 128: 8 waves of 64 x 32, direct loads, k-chunk 32
  static constexpr int TS = 128, WR = 2, WC = 4, KC = 32, DEPTH = 1, OCC = 2;
  static constexpr bool DMA = true;
  static constexpr int STAGES = 2;
};
template <> struct BigCfg<4> {   // 128: 8 waves of 64 x 32, direct loads, k-chunk 16, 2 workgroups per CU
  static constexpr int TS = 128, WR = 2, WC = 4, KC = 16, DEPTH = 1, OCC = 4;
  static constexpr bool DMA = true;
  static constexpr int STAGES = 2;
};
template <> struct BigCfg<5> {   // 128: 4 waves of 64 x 64, direct loads, k-chunk 16, 2 workgroups per CU
  static constexpr int TS = 128, WR = 2, WC = 2, KC = 16, DEPTH = 1, OCC = 2;
  static constexpr bool DMA = true;
  static constexpr int STAGES = 2;
};
template <> struct BigCfg<6> {   // 64: 4 waves of 32 x 32, direct loads, k-chunk 32, 2 workgroups per CU
  static constexpr int TS = 64, WR = 2, WC = 2, KC = 32, DEPTH = 1, OCC = 2;
  static constexpr bool DMA = true;
  static constexpr int STAGES = 2;
};
template <> struct BigCfg<7> {   // 64: 4 waves of 32 x 32, direct loads, k-chunk 16, 4 workgroups per CU
  static constexpr int TS = 64, WR = 2, WC = 2, KC = 16, DEPTH = 1, OCC = 4;
  static constexpr bool DMA = true;
  static constexpr int STAGES = 2;
};
template <> struct BigCfg<8> {   // 64: 4 waves of 32 x 32, direct loads, k-chunk 16, four LDS stages
  static constexpr int TS = 64, WR = 2, WC = 2, KC = 16, DEPTH = 1, OCC = 2;
  static constexpr bool DMA = true;
  static constexpr int STAGES = 4;
};
template <> struct BigCfg<9> {   // 64: 8 waves of 32 x 16, direct loads, k-chunk 16
  static constexpr int TS = 64, WR = 2, WC = 4, KC = 16, DEPTH = 1, OCC = 4;
  static constexpr bool DMA = true;
  static constexpr int STAGES = 2;
};
// Row length of a [k][row] LDS panel of a TS-row tile: 128 rows are padded by
// two; 64 rows stay unpadded so that one 1 KiB direct load fills two k-columns.
template <int TS> constexpr int pld() { return TS == 128 ? TS + 2 : TS; }
template <int V> constexpr int big_threads() { return 64 * BigCfg<V>::WR * BigCfg<V>::WC; }
template <int V> constexpr int big_lds() {
  return BigCfg<V>::STAGES * 2 * BigCfg<V>::KC * (BigCfg<V>::DMA ? pld<BigCfg<V>::TS>() : kBig + 2);
}

struct Seg {
  const double *A;
  const double *B;
  int ars, aks;                   // op(A)(r, k) = A[r*ars + k*aks]
  int brs, bks;                   // op(B)(c, k) = B[c*brs + k*bks];  product = op(A) op(B)^T
  int k0, k1;
  double alpha;
};

// TK_CHAIN: C = beta C - (A0 B0) A1^T (+ the plain product of seg[2], if any)
// with the 64-column intermediate A0 B0 kept in LDS (seg[0] = the first
// product, seg[1].A = A1).
// TK_LCHAIN: C = -A1 (S + A0 B0), A1 a lower-triangular diagonal tile (seg[1].A),
// S the tile at src (ld = ldc) if src is set, else 0.
enum TaskKind { TK_NONE = 0, TK_PRODUCT = 1, TK_COPY = 2, TK_ZERO = 3, TK_CHAIN = 4, TK_LCHAIN = 5 };

struct Task {
  int kind;
  int m, n;                       // output tile rows, cols
  double *C;
  long long ldc;
  double beta;                    // C = beta*C + sum_s alpha_s op(A_s) op(B_s)^T
  int nseg;
  Seg seg[3];
  int mirror;                     // 1: also store C^T at Cm (symmetric output); 2: zeros there
  int diagtile;                   // mirror: lower entries only
  double *Cm;
  int chol;                       // Cholesky + inverse of the result tile -> Lout
  double *Lout;
  long long ldl;
  double *ldsum;
  int row_off;
  double *Mout;                   // Cholesky tasks: also M = inv(L)^T inv(L) here (or null)
  int ti, tj;                     // 128-wide tiles: block coordinates of C (split-k scratch)
  const double *src;              // copy source; TK_LCHAIN: running-sum tile (ld = ldc)
  const double *init;             // TK_PRODUCT: the sum starts from this tile (ld = ldc), or 0
};

// Loads and stores through the global address space (global_load / global_store
// instead of flat ones, whose completion counter is shared with LDS traffic).
typedef __attribute__((address_space(1))) double gdouble;
__device__ __forceinline__ double gld(const double *p) {
  return *(const gdouble *)p;
}
__device__ __forceinline__ void gst(double *p, double v) { *(gdouble *)p = v; }

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
__device__ inline void set_seg(Seg &g, const double *A, int ars, int aks, const double *B, int brs,
                               int bks, int k0, int k1, double alpha) {
  g.A = A; g.ars = ars; g.aks = aks; g.B = B; g.brs = brs; g.bks = bks;
  g.k0 = k0; g.k1 = k1; g.alpha = alpha;
}

// Band of the coupling blocks (ItemDev::sbw).  Rows r >= r0 of S[t] and of
// X = S[t] inv(L_tt)^T are zero at k < r0 - sbw: band_lo is that bound
// rounded down to a multiple of 64 (0 when S is dense).  Rows r < r1 of S[t]
// are zero at k > r1 - 1 + sbw: band_hi is the exclusive bound rounded up to
// a multiple of 64, at most b.  Skipping those k ranges leaves out exact
// zeros only.
__device__ inline int band_lo(const ItemDev &it, int r0) {
  return it.sbw >= it.b ? 0 : (max(0, r0 - it.sbw) & ~(kTile - 1));
}
__device__ inline int band_hi(const ItemDev &it, int r1) {
  return it.sbw >= it.b ? it.b : min(it.b, ((r1 - 1 + it.sbw) / kTile + 1) * kTile);
}

// V_t = L_{t+1,t} inv(L_tt) and U_t = L_{A,t} inv(L_tt) of step t of the
// selected inversion: formed up front for every step (V, U) or step by step in
// the workspace (W2, W3).  V has no slot for the last step, whose V is never read.
__device__ inline const double *vmat(const ItemDev &it, int t) {
  return (it.V && t < it.nt - 1) ? it.V + (long long)t * it.b * it.b : it.W2;
}
__device__ inline const double *umat(const ItemDev &it, int t) {
  return it.U ? it.U + (long long)t * it.a * it.b : it.W3;
}

// Map (item, phase, t, p, local task q) to the work of one workgroup.
// SIDE >= 0: decode only the side phases that ride in a product-kernel launch
// of operand layout SIDE (0: the factorization's remainders, 2: the selected
// inversion's U and Sigma_R rows), or, SIDE = kFatOnly / kLeanOnly, only the
// phases of the Cholesky-capable / the lean tile kernel; the other cases
// compile to no code.
constexpr int kFatOnly = 100, kLeanOnly = 101;
#define SIDE_ONLY(keep)                                   \
  if constexpr (SIDE >= 0 && !(keep)) {                   \
    tk.kind = TK_NONE;                                    \
    return;                                               \
  }
template <int SIDE = -1>
__device__ __forceinline__ void decode(const ItemDev &it, int phase, int t, int p, int q, Task &tk) {
  const int b = it.b, a = it.a, nP = it.nP;
  const long long bb = (long long)b * b;
  const bool arrow = a > 0;
  const bool last = (t == it.nt - 1);
  tk.kind = TK_PRODUCT; tk.nseg = 0; tk.beta = 0.0; tk.mirror = 0; tk.diagtile = 0; tk.chol = 0;
  tk.Mout = nullptr;
  tk.Cm = nullptr; tk.Lout = nullptr; tk.ldsum = nullptr; tk.src = nullptr; tk.ldl = 0;
  tk.row_off = 0; tk.init = nullptr;
  double *Dt = dblk(it, t);
  double *St = it.S ? sblk(it, t) : nullptr;
  double *Rt = arrow ? rblk(it, t) : nullptr;
  switch (phase) {
    case PH_DIAG0: {
      SIDE_ONLY(SIDE == kFatOnly)
      tk.m = tk.n = tdim(b, 0);
      tk.C = Dt; tk.ldc = b; tk.beta = 1.0;
      tk.chol = 1; tk.Lout = Dt; tk.ldl = b;
      tk.ldsum = it.ldpart + (long long)t * nP; tk.row_off = tmap(it, t) * b;
      tk.Mout = it.Mp;
      return;
    }
    case PH_STEP:
    case PH_DIAGC:
    case PH_STEPF: {
      SIDE_ONLY(SIDE == kFatOnly || SIDE == kLeanOnly)
      // Tiles p-1 and p are full wherever they are used here (they precede a tile).
      // The batched step (PH_STEP with PH_DIAGC beside it) is left-looking:
      // column p+1 and its diagonal tile take every earlier panel in one
      // product here, and no trailing tile is touched before its column's
      // turn.  The fused step (few tiles) keeps the right-looking order with
      // the rest of panel p-1's update deferred to this launch.
      const bool left = phase != PH_STEPF;
      const int npan = nP - 1 - p;
      const int ncol = max(nP - 2 - p, 0);
      const int ndef = left ? 0 : (p >= 1) ? ncol * (ncol + 1) / 2 : min(ncol, 1);
      int i = -1, jc = p + 1;   // chained task for tile (i, jc)
      if (phase == PH_STEPF && p < nP - 1) {   // task 0 is the diagonal tile
        if (q == 0) i = p + 1;
        else --q;
      }
      if (i >= 0) {
      } else if (phase == PH_DIAGC) {
        i = p + 1;
      } else if (q < npan) {   // panel: W2(i,p) = A_ip inv(L_pp)^T
        const int ip = p + 1 + q;
        tk.m = tdim(b, ip); tk.n = kTile;
        tk.C = it.W2 + toff(b, ip, p); tk.ldc = b;
        set_seg(tk.seg[0], Dt + toff(b, ip, p), 1, b, Dt + toff(b, p, p), 1, b, 0, kTile, 1.0);
        tk.nseg = 1;
        return;
      } else if (q < npan + ncol) {
        i = p + 2 + (q - npan);
      } else if (q < npan + ncol + ndef) {
        // the rest of panel p-1's update: A_ij -= L_{i,p-1} L_{j,p-1}^T, p+1 < j <= i;
        // the diagonal tile of column p+2 also takes column p's term here (a
        // chained product), one step before it is factored
        int ii, jj;
        tri_decode(q - npan - ncol, ii, jj);
        const int id = p + 2 + ii, jd = p + 2 + jj;
        if (id == p + 2) {
          i = p + 2;
          jc = p + 2;
        } else {
          tk.m = tdim(b, id); tk.n = tdim(b, jd);
          tk.C = Dt + toff(b, id, jd); tk.ldc = b; tk.beta = 1.0;
          set_seg(tk.seg[0], it.W2 + toff(b, id, p - 1), 1, b, it.W2 + toff(b, jd, p - 1), 1, b, 0,
                  kTile, -1.0);
          tk.nseg = 1;
          return;
        }
      } else if (q < npan + ncol + ndef + p) {
        // row p of X = inv(L_tt): X_pj = -X_pp sum_{m=j}^{p-1} L_pm X_mj, j < p.
        // The fused step (few tiles: latency matters) keeps the running sum
        // T_pj = sum_{m=j}^{p-2} L_pm X_mj in W1 (none for j = p-1) and adds the
        // last term here; the batched step takes the whole sum in one product
        // (throughput matters: no partial sums through memory).  X is built in
        // place of D[t]: its columns j < p are no longer needed by the
        // factorization (L is in W2); the tile (j,p) above the diagonal is set
        // to zero at the same time.
        const int j = q - npan - ncol - ndef;
        const bool sums = phase == PH_STEPF;
        tk.kind = TK_LCHAIN;
        tk.m = tdim(b, p); tk.n = kTile;
        tk.C = Dt + toff(b, p, j); tk.ldc = b;
        tk.mirror = 2; tk.Cm = Dt + toff(b, j, p);
        set_seg(tk.seg[0], it.W2 + (long long)p * kTile, 1, b, Dt + (long long)j * kTile * b, b, 1,
                sums ? (p - 1) * kTile : j * kTile, p * kTile, 1.0);
        set_seg(tk.seg[1], Dt + toff(b, p, p), 1, b, nullptr, 0, 0, 0, tdim(b, p), -1.0);
        tk.nseg = 1;
        tk.src = (sums && j < p - 1) ? it.W1 + toff(b, p, j) : nullptr;
        return;
      } else {
        // (fused step) running sums of the later rows: T_rj (+)= L_{r,p-1} X_{p-1,j}
        // for r > p, j < p (the term m = p-1, ready once row p-1 of X is)
        const int e = q - npan - ncol - ndef - p;
        const int r = p + 1 + e / p, j = e % p;
        tk.m = tdim(b, r); tk.n = kTile;
        tk.C = it.W1 + toff(b, r, j); tk.ldc = b; tk.beta = (j == p - 1) ? 0.0 : 1.0;
        set_seg(tk.seg[0], it.W2 + (long long)r * kTile, 1, b, Dt + (long long)j * kTile * b, b, 1,
                (p - 1) * kTile, p * kTile, 1.0);
        tk.nseg = 1;
        return;
      }
      // column p+1 (and, right-looking, the diagonal tile of column p+2):
      // right-looking, A_{i,jc} -= L_{i,p-1} L_{jc,p-1}^T + L_{i,p} L_{jc,p}^T
      // (the diagonal tile factored in this step took its column p-1 term in
      // the previous one); left-looking, A_{i,jc} -= sum_{m <= p} L_{i,m} L_{jc,m}^T.
      // The fused step forms L_{i,p} = A_ip X_pp^T and L_{jc,p} in the task
      // (X_pp = inv(L_pp) is in place in D[t]); the batched one takes
      // (A_ip M_p) A_{jc,p}^T with M_p = X_pp^T X_pp = inv(A_pp), which the
      // diagonal task of the previous step leaves in Mp
      const bool fac = (i == p + 1 && jc == p + 1);
      tk.kind = TK_CHAIN;
      tk.m = tdim(b, i); tk.n = tdim(b, jc);
      tk.C = Dt + toff(b, i, jc); tk.ldc = b; tk.beta = 1.0;
      if (phase == PH_STEPF) {
        set_seg(tk.seg[0], Dt + toff(b, i, p), 1, b, Dt + toff(b, p, p), 1, b, 0, kTile, 1.0);
        set_seg(tk.seg[1], Dt + toff(b, jc, p), 1, b, Dt + toff(b, p, p), 1, b, 0, kTile, -1.0);
      } else {
        set_seg(tk.seg[0], Dt + toff(b, i, p), 1, b, it.Mp + (long long)(p & 1) * kTile * kTile,
                kTile, 1, 0, kTile, 1.0);
        set_seg(tk.seg[1], Dt + toff(b, jc, p), 1, b, nullptr, 0, 0, 0, kTile, -1.0);
      }
      if (left && p >= 1)
        // panels 0..p-1 of L_tt (in W2) in one product of k = 64 p
        set_seg(tk.seg[2], it.W2 + (long long)i * kTile, 1, b, it.W2 + (long long)jc * kTile, 1, b, 0,
                p * kTile, -1.0);
      else if (p >= 1 && !fac)
        set_seg(tk.seg[2], it.W2 + toff(b, i, p - 1), 1, b, it.W2 + toff(b, jc, p - 1), 1, b, 0,
                kTile, -1.0);
      else
        set_seg(tk.seg[2], nullptr, 1, b, nullptr, 1, b, 0, 0, -1.0);
      tk.nseg = 1;
      if (fac) {
        tk.chol = 1; tk.Lout = Dt + toff(b, i, i); tk.ldl = b;
        tk.ldsum = it.ldpart + (long long)t * nP + i; tk.row_off = tmap(it, t) * b + i * kTile;
        tk.Mout = (phase == PH_STEPF) ? nullptr : it.Mp + (long long)((p + 1) & 1) * kTile * kTile;
      }
      return;
    }
    case PH_OFFDIAG_X: {
      SIDE_ONLY(SIDE == kLeanOnly)
      // k runs to the end of tile column j: the longest tiles first
      // (X = S[t] inv(L_tt)^T: k <= the last column of tile j, and within S's band)
      const int j = nP - 1 - q / nP, i = q % nP;
      tk.m = tdim(b, i); tk.n = tdim(b, j);
      tk.C = it.W2 + toff(b, i, j); tk.ldc = b;
      set_seg(tk.seg[0], St + (long long)i * kTile, 1, b, Dt + (long long)j * kTile, 1, b,
              band_lo(it, i * kTile), min(min(b, (j + 1) * kTile), band_hi(it, i * kTile + tk.m)),
              1.0);
      tk.nseg = 1;
      return;
    }
    case PH_OFFDIAG: {
      SIDE_ONLY(SIDE == 0 || SIDE == kLeanOnly)
      int idx = q;
      if (arrow) {
        if (idx < nP) {
          const int j = idx;
          tk.m = a; tk.n = tdim(b, j);
          tk.C = it.W3 + (long long)j * kTile * a; tk.ldc = a;
          set_seg(tk.seg[0], Rt, 1, a, Dt + (long long)j * kTile, 1, b, 0, min(b, (j + 1) * kTile),
                  1.0);
          tk.nseg = 1;
          return;
        }
        idx -= nP;
      }
      tk.kind = TK_NONE;
      return;
    }
    case PH_SCHUR_X: {
      SIDE_ONLY(SIDE == kLeanOnly)
      int i, j;
      tri_decode(q, i, j);   // i >= j: the rows of tile i bound the nonzero k of both
      tk.m = tdim(b, i); tk.n = tdim(b, j);
      tk.C = dblk(it, t + 1) + toff(b, i, j); tk.ldc = b; tk.beta = 1.0;
      set_seg(tk.seg[0], it.W2 + (long long)i * kTile, 1, b, it.W2 + (long long)j * kTile, 1, b,
              band_lo(it, i * kTile), b, -1.0);
      tk.nseg = 1;
      return;
    }
    case PH_SCHUR: {
      SIDE_ONLY(SIDE == 0 || SIDE == kLeanOnly)
      int idx = q;
      if (!last) {
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
            tk.C = rblk(it, t + 1) + (long long)j * kTile * a; tk.ldc = a;
            tk.beta = 1.0;
            set_seg(tk.seg[0], it.W3, 1, a, it.W2 + (long long)j * kTile, 1, b,
                    band_lo(it, j * kTile), b, -1.0);
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
      SIDE_ONLY(SIDE == kFatOnly)
      tk.m = tk.n = a;
      tk.C = it.T; tk.ldc = a; tk.beta = 1.0;
      tk.chol = 1; tk.Lout = it.T; tk.ldl = a;
      tk.ldsum = it.ldpart + (long long)it.nt * nP; tk.row_off = it.nt * b;
      return;
    }
    case PH_SI_INIT: {
      SIDE_ONLY(SIDE == kLeanOnly)
      tk.m = tk.n = a;
      tk.C = it.ST; tk.ldc = a;
      set_seg(tk.seg[0], it.T, a, 1, it.T, a, 1, 0, a, 1.0);
      tk.nseg = 1;
      return;
    }
    case PH_SI_VU_X: {
      SIDE_ONLY(SIDE == kLeanOnly)
      // k starts at tile column j: the longest tiles first
      const int j = q / nP, i = q % nP;
      tk.m = tdim(b, i); tk.n = tdim(b, j);
      tk.C = it.W2 + toff(b, i, j); tk.ldc = b;
      set_seg(tk.seg[0], St + (long long)i * kTile, 1, b, Dt + (long long)j * kTile * b, b, 1,
              max(j * kTile, band_lo(it, i * kTile)), b, 1.0);
      tk.nseg = 1;
      return;
    }
    case PH_SI_VU: {
      SIDE_ONLY(SIDE == 2 || SIDE == kLeanOnly)
      const int j = q;
      tk.m = a; tk.n = tdim(b, j);
      tk.C = it.W3 + (long long)j * kTile * a; tk.ldc = a;
      set_seg(tk.seg[0], Rt, 1, a, Dt + (long long)j * kTile * b, b, 1, j * kTile, b, 1.0);
      tk.nseg = 1;
      return;
    }
    case PH_SI_VU_B: {
      SIDE_ONLY(SIDE == kLeanOnly)
      // as PH_SI_VU_X for every step tt < nt-1: q runs over (tt, tile)
      const int per = nP * nP, tt = q / per, r = q - tt * per;
      const int j = r / nP, i = r % nP;
      const double *Dq = dblk(it, tt), *Sq = sblk(it, tt);
      tk.m = tdim(b, i); tk.n = tdim(b, j);
      tk.C = it.V + (long long)tt * bb + toff(b, i, j); tk.ldc = b;
      set_seg(tk.seg[0], Sq + (long long)i * kTile, 1, b, Dq + (long long)j * kTile * b, b, 1,
              max(j * kTile, band_lo(it, i * kTile)), b, 1.0);
      tk.nseg = 1;
      return;
    }
    case PH_SI_G_B: {
      SIDE_ONLY(SIDE == kLeanOnly)
      // inv(L_tt)^T inv(L_tt) of every step tt, lower tiles (the first term of
      // PH_SI_SD_X, in full tiles: no mirror)
      const int per = nP * (nP + 1) / 2, tt = q / per;
      int i, j;
      tri_decode(q - tt * per, i, j);
      const double *Dq = dblk(it, tt);
      tk.m = tdim(b, i); tk.n = tdim(b, j);
      tk.C = it.G + (long long)tt * bb + toff(b, i, j); tk.ldc = b;
      set_seg(tk.seg[0], Dq + (long long)i * kTile * b, b, 1, Dq + (long long)j * kTile * b, b, 1,
              i * kTile, b, 1.0);
      tk.nseg = 1;
      return;
    }
    case PH_SI_U_B: {
      SIDE_ONLY(SIDE == 2 || SIDE == kLeanOnly)
      // as PH_SI_VU for every step tt
      const int tt = q / nP, j = q % nP;
      const double *Dq = dblk(it, tt);
      tk.m = a; tk.n = tdim(b, j);
      tk.C = it.U + (long long)tt * a * b + (long long)j * kTile * a; tk.ldc = a;
      set_seg(tk.seg[0], rblk(it, tt), 1, a, Dq + (long long)j * kTile * b, b, 1,
              j * kTile, b, 1.0);
      tk.nseg = 1;
      return;
    }
    case PH_SI_SR_X: {
      SIDE_ONLY(SIDE == kLeanOnly)
      const int i = q / nP, j = q % nP;
      double *SDn = sig_D(it, t + 1);
      tk.m = tdim(b, i); tk.n = tdim(b, j);
      tk.C = sig_S(it, t) + toff(b, i, j); tk.ldc = b;
      set_seg(tk.seg[0], SDn + (long long)i * kTile, 1, b, vmat(it, t) + (long long)j * kTile * b, b,
              1, 0, b, -1.0);
      tk.nseg = 1;
      if (arrow) {
        set_seg(tk.seg[1], sig_R(it, t + 1) + (long long)i * kTile * a, a, 1,
                umat(it, t) + (long long)j * kTile * a, a, 1, 0, a, -1.0);
        tk.nseg = 2;
      }
      return;
    }
    case PH_SI_SR: {
      SIDE_ONLY(SIDE == 2 || SIDE == kLeanOnly)
      const int j = q;
      tk.m = a; tk.n = tdim(b, j);
      tk.C = sig_R(it, t) + (long long)j * kTile * a; tk.ldc = a;
      // every segment has a fixed slot (an empty one when absent), so that the
      // task never needs an indexed segment
      set_seg(tk.seg[0], it.ST, 1, a, umat(it, t) + (long long)j * kTile * a, a, 1, 0, a, -1.0);
      set_seg(tk.seg[1], sig_R(it, t + 1), 1, a, vmat(it, t) + (long long)j * kTile * b, b, 1, 0,
              last ? 0 : b, -1.0);
      tk.nseg = 2;
      return;
    }
    case PH_SI_SD_X: {
      SIDE_ONLY(SIDE == kLeanOnly)
      int i, j;
      tri_decode(q, i, j);
      double *SDt = sig_D(it, t);
      tk.m = tdim(b, i); tk.n = tdim(b, j);
      tk.C = SDt + toff(b, i, j); tk.ldc = b;
      tk.mirror = 1; tk.Cm = SDt + toff(b, j, i); tk.diagtile = (i == j);
      // fixed slots: LinvT Linv, then - Sigma_S^T V, then - Sigma_R^T U (empty when absent);
      // with G the first term is there already and the sum starts from it
      set_seg(tk.seg[0], Dt + (long long)i * kTile * b, b, 1, Dt + (long long)j * kTile * b, b, 1,
              it.G ? 0 : i * kTile, it.G ? 0 : b, 1.0);
      if (it.G) tk.init = it.G + (long long)t * bb + toff(b, i, j);
      set_seg(tk.seg[1], sig_S(it, t) + (long long)i * kTile * b, b, 1,
              vmat(it, t) + (long long)j * kTile * b, b, 1, 0, last ? 0 : b, -1.0);
      set_seg(tk.seg[2], sig_R(it, t) + (long long)i * kTile * a, a, 1,
              umat(it, t) + (long long)j * kTile * a, a, 1, 0, a, -1.0);
      tk.nseg = 3;
      return;
    }
    default:
      tk.kind = TK_NONE;
      return;
  }
}
#undef SIDE_ONLY

// Map (item, product phase, t, local task q) to one TS x TS output tile (TS =
// 64 or 128).  For 128 the k ranges are those of the 64-tile form widened to
// the big tile; the extra range only meets entries that are stored as zeros
// (inv(L_tt) and the factor blocks keep zeros above their diagonal).
template <int TS>
__device__ __forceinline__ long long boff(int b, int I, int J) {
  return (long long)I * TS + (long long)J * TS * b;
}
template <int TS>
__device__ __forceinline__ int bdim(int n, int I) { return min(TS, n - I * TS); }

// A launch of the product kernel decodes only the phases of its operand
// layout (LAY, as big_layouts assigns them): the other cases compile to no
// code, which keeps the kernel's registers to what its own phases need.
// LAY < 0 (the split-k reduction) decodes every phase.
#define LAY_ONLY(l)                                       \
  if constexpr (!(LAY < 0 || LAY == (l))) {               \
    tk.kind = TK_NONE;                                    \
    return;                                               \
  }
template <int TS, int LAY = -1>
__device__ __forceinline__ void decode_big(const ItemDev &it, int phase, int t, int q, Task &tk) {
  const int b = it.b, a = it.a, nQ = (it.b + TS - 1) / TS;
  const long long bb = (long long)b * b;
  const bool arrow = a > 0;
  const bool last = (t == it.nt - 1);
  tk.kind = TK_PRODUCT; tk.nseg = 0; tk.beta = 0.0; tk.mirror = 0; tk.diagtile = 0; tk.chol = 0;
  tk.Mout = nullptr;
  tk.Cm = nullptr; tk.Lout = nullptr; tk.ldsum = nullptr; tk.src = nullptr; tk.ldl = 0;
  tk.row_off = 0; tk.init = nullptr;
  double *Dt = dblk(it, t);
  double *St = it.S ? sblk(it, t) : nullptr;
  int I, J;
  switch (phase) {
    case PH_OFFDIAG_X:
      LAY_ONLY(0)
      // k runs to the end of tile column J: tiles of the last columns (the
      // longest) first, so that the short ones fill the end of the launch
      J = nQ - 1 - q / nQ; I = q % nQ;
      tk.m = bdim<TS>(b, I); tk.n = bdim<TS>(b, J); tk.ti = I; tk.tj = J;
      tk.C = it.W2 + boff<TS>(b, I, J); tk.ldc = b;
      set_seg(tk.seg[0], St + (long long)I * TS, 1, b, Dt + (long long)J * TS, 1, b,
              band_lo(it, I * TS), min(min(b, (J + 1) * TS), band_hi(it, I * TS + tk.m)), 1.0);
      tk.nseg = 1;
      return;
    case PH_SCHUR_X:
      LAY_ONLY(0)
      tri_decode(q, I, J);
      tk.m = bdim<TS>(b, I); tk.n = bdim<TS>(b, J); tk.ti = I; tk.tj = J;
      tk.C = dblk(it, t + 1) + boff<TS>(b, I, J); tk.ldc = b; tk.beta = 1.0;
      set_seg(tk.seg[0], it.W2 + (long long)I * TS, 1, b, it.W2 + (long long)J * TS, 1, b,
              band_lo(it, I * TS), b, -1.0);
      tk.nseg = 1;
      return;
    case PH_SI_VU_X:
      LAY_ONLY(2)
      // k starts at tile column J: the first columns (the longest) first
      J = q / nQ; I = q % nQ;
      tk.m = bdim<TS>(b, I); tk.n = bdim<TS>(b, J); tk.ti = I; tk.tj = J;
      tk.C = it.W2 + boff<TS>(b, I, J); tk.ldc = b;
      set_seg(tk.seg[0], St + (long long)I * TS, 1, b, Dt + (long long)J * TS * b, b, 1,
              max(J * TS, band_lo(it, I * TS)), b, 1.0);
      tk.nseg = 1;
      return;
    case PH_SI_VU_B: {
      LAY_ONLY(2)
      // as PH_SI_VU_X for every step tt < nt-1: q runs over (tt, tile)
      const int per = nQ * nQ, tt = q / per, r = q - tt * per;
      J = r / nQ; I = r % nQ;
      const double *Dq = dblk(it, tt), *Sq = sblk(it, tt);
      tk.m = bdim<TS>(b, I); tk.n = bdim<TS>(b, J); tk.ti = I; tk.tj = J;
      tk.C = it.V + (long long)tt * bb + boff<TS>(b, I, J); tk.ldc = b;
      set_seg(tk.seg[0], Sq + (long long)I * TS, 1, b, Dq + (long long)J * TS * b, b, 1,
              max(J * TS, band_lo(it, I * TS)), b, 1.0);
      tk.nseg = 1;
      return;
    }
    case PH_SI_SR_X:
      LAY_ONLY(2)
      I = q / nQ; J = q % nQ;
      tk.m = bdim<TS>(b, I); tk.n = bdim<TS>(b, J); tk.ti = I; tk.tj = J;
      tk.C = sig_S(it, t) + boff<TS>(b, I, J); tk.ldc = b;
      set_seg(tk.seg[0], sig_D(it, t + 1) + (long long)I * TS, 1, b,
              vmat(it, t) + (long long)J * TS * b, b, 1, 0, b, -1.0);
      tk.nseg = 1;
      if (arrow) {
        set_seg(tk.seg[1], sig_R(it, t + 1) + (long long)I * TS * a, a, 1,
                umat(it, t) + (long long)J * TS * a, a, 1, 0, a, -1.0);
        tk.nseg = 2;
      }
      return;
    case PH_SI_G_B: {
      LAY_ONLY(3)
      // inv(L_tt)^T inv(L_tt) of every step tt, lower tiles (full tiles: no mirror)
      const int per = nQ * (nQ + 1) / 2, tt = q / per;
      tri_decode(q - tt * per, I, J);
      const double *Dq = dblk(it, tt);
      tk.m = bdim<TS>(b, I); tk.n = bdim<TS>(b, J); tk.ti = I; tk.tj = J;
      tk.C = it.G + (long long)tt * bb + boff<TS>(b, I, J); tk.ldc = b;
      set_seg(tk.seg[0], Dq + (long long)I * TS * b, b, 1, Dq + (long long)J * TS * b, b, 1, I * TS,
              b, 1.0);
      tk.nseg = 1;
      return;
    }
    case PH_SI_SD_X: {
      LAY_ONLY(3)
      tri_decode(q, I, J);
      double *SDt = sig_D(it, t);
      tk.m = bdim<TS>(b, I); tk.n = bdim<TS>(b, J); tk.ti = I; tk.tj = J;
      tk.C = SDt + boff<TS>(b, I, J); tk.ldc = b;
      tk.mirror = 1; tk.Cm = SDt + boff<TS>(b, J, I); tk.diagtile = (I == J);
      set_seg(tk.seg[0], Dt + (long long)I * TS * b, b, 1, Dt + (long long)J * TS * b, b, 1,
              it.G ? 0 : I * TS, it.G ? 0 : b, 1.0);
      if (it.G) tk.init = it.G + (long long)t * bb + boff<TS>(b, I, J);
      set_seg(tk.seg[1], sig_S(it, t) + (long long)I * TS * b, b, 1,
              vmat(it, t) + (long long)J * TS * b, b, 1, 0, last ? 0 : b, -1.0);
      set_seg(tk.seg[2], sig_R(it, t) + (long long)I * TS * a, a, 1,
              umat(it, t) + (long long)J * TS * a, a, 1, 0, a, -1.0);
      tk.nseg = 3;
      return;
    }
    default:
      tk.kind = TK_NONE;
      return;
  }
}
#undef LAY_ONLY

// Global -> register staging of rows [0, rows) x k in [kc, min(kc+KC, k1)) of op(X)
// for a panel of ROWS rows, NT threads.  Addresses are clamped into range so
// that every load is unconditional and all of them stay in flight together;
// masking and scaling happen at the LDS store.
// Element q of a thread's share of a KC x ROWS chunk: row r0 + q*dr, k k0 + q*dk.
// Row-contiguous operands give each thread one row and a run of k (coalesced
// along rows); k-contiguous ones give each thread one k and a run of rows.
template <int KC, int ROWS, int NT>
struct ChunkMap {
  int r0, dr, k0, dk;
  __device__ __forceinline__ ChunkMap(bool rows_contig) {
    static_assert(NT % ROWS == 0 && NT % KC == 0, "chunk map needs NT to be a multiple");
    const int tid = threadIdx.x;
    r0 = rows_contig ? tid % ROWS : tid / KC;
    dr = rows_contig ? 0 : NT / KC;
    k0 = rows_contig ? tid / ROWS : tid % KC;
    dk = rows_contig ? NT / ROWS : 0;
  }
};

// Raw loads of one KC x ROWS chunk of op(X)(r, k) = X[r*rs + k*ks] into
// registers.  Addresses are clamped into range so that every load is
// unconditional and all of them stay in flight together; masking and scaling
// happen at the LDS store.
template <int KC, int ROWS, int NT>
__device__ __forceinline__ void gload(double (&r)[KC * ROWS / NT], const double *X, int rs, int ks,
                                      int rows, int kc, int k1) {
  constexpr int NE = KC * ROWS / NT;
  const ChunkMap<KC, ROWS, NT> cm(rs == 1);
  const int rmax = rows - 1, kmax = k1 - 1;
#pragma unroll
  for (int q = 0; q < NE; ++q) {
    const int rr = min(cm.r0 + q * cm.dr, rmax), kk = min(kc + cm.k0 + q * cm.dk, kmax);
    r[q] = gld(X + (long long)rr * rs + (long long)kk * ks);
  }
}

// Register -> LDS panel P[k][row] (row length ROWS + 2), zeroing out-of-range
// entries and applying alpha.
template <int KC, int ROWS, int NT>
__device__ __forceinline__ void sstore(double *P, const double (&r)[KC * ROWS / NT], bool rows_contig,
                                       int rows, int kc, int k1, double alpha) {
  constexpr int NE = KC * ROWS / NT;
  constexpr int LD = ROWS + 2;
  const ChunkMap<KC, ROWS, NT> cm(rows_contig);
#pragma unroll
  for (int q = 0; q < NE; ++q) {
    const int rr = cm.r0 + q * cm.dr, k = cm.k0 + q * cm.dk;
    P[k * LD + rr] = (rr < rows && kc + k < k1) ? alpha * r[q] : 0.0;
  }
}

// Value of segment 0, 1 or 2 (arguments by value, so the choice is a select of
// registers and never an indexed access into the task).
template <class T>
__device__ __forceinline__ T pick3(bool s1, bool s2, T v0, T v1, T v2) {
  return s2 ? v2 : (s1 ? v1 : v0);
}

// Geometry of the chunk held in the staging registers.
struct ChunkInfo {
  bool fa, fb;     // operand rows contiguous
  int kc, k1;
  double alpha;
};

// acc += sum over segments of op(A) op(B)^T for an output tile of ROWS x ROWS
// computed by WR x WC waves; wave (wr, wc) owns rows wr*ROWS/WR .. and columns
// wc*ROWS/WC .., i.e. MR x MC MFMA blocks of 16 x 16.  LDS panels are
// double-buffered with one barrier per chunk.  With DEPTH = 1 the next chunk
// is fetched into registers while the current one feeds the matrix cores; with
// DEPTH = 2 two register sets alternate so that the loads of chunk c + 2 are
// issued while chunk c is multiplied and have two chunk-times to arrive.
// Chunks are numbered across the segments; segment fields are only indexed by
// constants so the task stays in registers.
template <int KC, int ROWS, int WR, int WC, int DEPTH = 1, bool SHORT = false>
__device__ __forceinline__ void run_product(const Task &tk, double *smem,
                                            d4 (&acc)[ROWS / WR / 16][ROWS / WC / 16],
                                            int part = 0, int nparts = 1) {
  constexpr int NT = 64 * WR * WC;
  constexpr int NE = KC * ROWS / NT;
  constexpr int LD = ROWS + 2;
  constexpr int MR = ROWS / WR / 16, MC = ROWS / WC / 16;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w / WC, wc = w % WC;
  const int n0 = (tk.nseg > 0 && tk.seg[0].k1 > tk.seg[0].k0) ? (tk.seg[0].k1 - tk.seg[0].k0 + KC - 1) / KC : 0;
  const int n1 = (tk.nseg > 1 && tk.seg[1].k1 > tk.seg[1].k0) ? (tk.seg[1].k1 - tk.seg[1].k0 + KC - 1) / KC : 0;
  const int n2 = (tk.nseg > 2 && tk.seg[2].k1 > tk.seg[2].k0) ? (tk.seg[2].k1 - tk.seg[2].k0 + KC - 1) / KC : 0;
  // this workgroup's share of the chunks (all of them unless the k range is split)
  const int all = n0 + n1 + n2;
  const int cb = (int)((long long)all * part / nparts), ce = (int)((long long)all * (part + 1) / nparts);
  if (ce <= cb) return;
  // chunk c of the concatenated segments; the segment's fields are picked
  // with uniform selects so that a single copy of the load code exists
  auto fetch = [&](int c, double (&ra)[NE], double (&rb)[NE], ChunkInfo &ci) {
    const bool s1 = c >= n0, s2 = c >= n0 + n1;
    const double *A = pick3(s1, s2, tk.seg[0].A, tk.seg[1].A, tk.seg[2].A);
    const double *B = pick3(s1, s2, tk.seg[0].B, tk.seg[1].B, tk.seg[2].B);
    const int ars = pick3(s1, s2, tk.seg[0].ars, tk.seg[1].ars, tk.seg[2].ars);
    const int aks = pick3(s1, s2, tk.seg[0].aks, tk.seg[1].aks, tk.seg[2].aks);
    const int brs = pick3(s1, s2, tk.seg[0].brs, tk.seg[1].brs, tk.seg[2].brs);
    const int bks = pick3(s1, s2, tk.seg[0].bks, tk.seg[1].bks, tk.seg[2].bks);
    const int k0 = pick3(s1, s2, tk.seg[0].k0, tk.seg[1].k0, tk.seg[2].k0);
    const int k1 = pick3(s1, s2, tk.seg[0].k1, tk.seg[1].k1, tk.seg[2].k1);
    const int cs = c - (s2 ? n0 + n1 : (s1 ? n0 : 0));
    const int kc = k0 + cs * KC;
    gload<KC, ROWS, NT>(ra, A, ars, aks, tk.m, kc, k1);
    gload<KC, ROWS, NT>(rb, B, brs, bks, tk.n, kc, k1);
    ci.fa = ars == 1;
    ci.fb = brs == 1;
    ci.kc = kc;
    ci.k1 = k1;
    ci.alpha = pick3(s1, s2, tk.seg[0].alpha, tk.seg[1].alpha, tk.seg[2].alpha);
  };
  auto stage = [&](double *dst, const double (&ra)[NE], const double (&rb)[NE], const ChunkInfo &ci) {
    sstore<KC, ROWS, NT>(dst, ra, ci.fa, tk.m, ci.kc, ci.k1, ci.alpha);
    sstore<KC, ROWS, NT>(dst + KC * LD, rb, ci.fb, tk.n, ci.kc, ci.k1, 1.0);
  };
  auto compute = [&](const double *As) {
    const double *Bs = As + KC * LD;
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      const int kr = (kk + (lane >> 4)) * LD;
      double av[MR], bv[MC];
#pragma unroll
      for (int x = 0; x < MR; ++x) av[x] = As[kr + wr * (ROWS / WR) + x * 16 + (lane & 15)];
#pragma unroll
      for (int x = 0; x < MC; ++x) bv[x] = Bs[kr + wc * (ROWS / WC) + x * 16 + (lane & 15)];
#pragma unroll
      for (int mi = 0; mi < MR; ++mi)
#pragma unroll
        for (int nj = 0; nj < MC; ++nj)
          acc[mi][nj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[mi], bv[nj], acc[mi][nj], 0, 0, 0);
    }
  };
  double *buf0 = smem, *buf1 = smem + 2 * KC * LD;
  double ra0[NE], rb0[NE];
  ChunkInfo ci0;
  if constexpr (DEPTH == 1) {
    fetch(cb, ra0, rb0, ci0);
    stage(buf0, ra0, rb0, ci0);
    __syncthreads();
    for (int c = cb; c < ce; ++c) {
      const int cur = (c - cb) & 1;
      const bool has_next = c + 1 < ce;
      fetch(min(c + 1, ce - 1), ra0, rb0, ci0);
      compute(cur ? buf1 : buf0);
      if (has_next) stage(cur ? buf0 : buf1, ra0, rb0, ci0);
      __syncthreads();
    }
  } else {
    // The loads are issued unconditionally (past the end they re-read the last
    // chunk, which stays unused) so that every wait on a register set counts
    // exactly the loads issued after it and leaves them in flight.
    double ra1[NE], rb1[NE];
    ChunkInfo ci1;
    const int last = ce - 1;
    fetch(cb, ra0, rb0, ci0);
    fetch(min(cb + 1, last), ra1, rb1, ci1);
    stage(buf0, ra0, rb0, ci0);
    __syncthreads();
    if (SHORT && ce - cb <= 2) {
      // one or two chunks: nothing more to fetch; chunk 0 is multiplied while
      // chunk 1 lands (SHORT: only where the registers allow the extra path)
      compute(buf0);
      if (ce - cb == 2) {
        stage(buf1, ra1, rb1, ci1);
        __syncthreads();
        compute(buf1);
      }
      __syncthreads();
      return;
    }
    // invariant at the top: buf0 holds chunk c, set 1 holds (or awaits) chunk c + 1
    for (int c = cb; c < ce; c += 2) {
      fetch(min(c + 2, last), ra0, rb0, ci0);
      compute(buf0);
      if (c + 1 < ce) stage(buf1, ra1, rb1, ci1);
      __syncthreads();
      if (c + 1 >= ce) break;
      fetch(min(c + 3, last), ra1, rb1, ci1);
      compute(buf1);
      if (c + 2 < ce) stage(buf0, ra0, rb0, ci0);
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// Direct-to-LDS staging for the product kernel (TS = 64 or 128 rows)
// ---------------------------------------------------------------------------
// global_load_lds_dwordx4 (dword) moves 16 (4) bytes per lane from any global
// address straight into LDS at M0 + 16 (4) * lane, with no registers and no
// LDS store instructions in between.  Each chunk of KC k-values of an operand
// lands in one of two layouts, fixed per launch and operand:
//   P[k][row] (row length pld<TS>), for operands whose rows are contiguous
//     (op(X)(r, k) = X[r + k*ks]): one wave instruction fills 1 KiB, one
//     k-column of 128 rows or two of 64.
//   Q[row][k] (row length KC, no padding), for operands whose k runs are
//     contiguous (op(X)(r, k) = X[r*rs + k]): the 16-byte slot j of row r
//     holds k = 2(j ^ qswz(r)), 2(j ^ qswz(r)) + 1, which spreads the 16-byte
//     reads of consecutive rows over the banks.
// Out-of-range k reads a 16-byte block of zeros; rows past the tile's end
// repeat the last row (those rows of the product are never stored).
// Global addresses need only dword alignment, which every double satisfies.
__device__ double g_dma_zeros[4];

typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) void glb_void_t;
__device__ __forceinline__ void dma16(const void *src, double *dst) {
  __builtin_amdgcn_global_load_lds((glb_void_t *)src, (lds_void_t *)dst, 16, 0, 0);
}
__device__ __forceinline__ void dma4(const void *src, double *dst) {
  __builtin_amdgcn_global_load_lds((glb_void_t *)src, (lds_void_t *)dst, 4, 0, 0);
}

// Slot permutation of Q row r (r16 = r mod 16): KC = 16 has 8 slots of 16
// bytes per row, KC = 32 has 16.  With these the 16-byte reads of the matrix
// loop run free of LDS bank conflicts (rocprofv3 SQ_LDS_BANK_CONFLICT = 0 on
// gfx950; (r mod 8) xor ((r / 8) mod 2) for KC = 16 gave one conflict cycle
// per matrix instruction, without a measurable change in time).
template <int KC>
__device__ __forceinline__ int qswz(int r16) {
  return KC == 16 ? (r16 & 7) : (r16 & 15);
}

// Issue the direct loads of rows [0, rows) x k in [kc, kc + KC) of
// op(X)(r, k) = X[r*rs + k*ks] into dst in layout Q (QL) or P for a panel of
// TS rows; wave w of NW takes every NW-th instruction.  16-byte pieces where
// the operand's contiguous direction matches the layout (and, in P, an even
// row count keeps the last pair inside the operand; in Q, k-pairs do not
// straddle k1), else 4-byte pieces with any strides.
template <int KC, int NW, bool QL, int TS>
__device__ __forceinline__ void dma_operand(const double *X, int rs, int ks, int rows, int kc,
                                            int k1, double *dst, int w, int lane) {
  constexpr int LD = pld<TS>();
  constexpr int SPR = KC / 2;          // 16-byte slots per Q row
  constexpr int CPI = 128 / TS;        // k-columns per 16-byte P instruction
  constexpr int DPC = TS / 32;         // 4-byte instructions per P k-column
  const double *zero = g_dma_zeros;
  if constexpr (!QL) {
    if (rs == 1 && (rows & 1) == 0) {
      const int r = min(2 * (lane % (TS / 2)), rows - 2), kl = lane / (TS / 2);
#pragma unroll 1
      for (int i = 0; i < KC / CPI / NW; ++i) {
        const int h = w + i * NW, k = kc + h * CPI + kl;
        dma16(k < k1 ? X + r + (long long)k * ks : zero, dst + h * CPI * LD);
      }
    } else {
#pragma unroll 1
      for (int i = 0; i < DPC * KC / NW; ++i) {
        const int h = w + i * NW, kk = h / DPC, qd = h % DPC;
        const int d = qd * 64 + lane, r = min(d >> 1, rows - 1), k = kc + kk;
        const char *src = (const char *)(X + (long long)r * rs + (long long)k * ks) + (d & 1) * 4;
        dma4(k < k1 ? (const void *)src : (const void *)zero, dst + kk * LD + qd * 32);
      }
    }
  } else {
    if (ks == 1 && (kc + KC <= k1 || ((k1 - kc) & 1) == 0)) {
#pragma unroll 1
      for (int i = 0; i < KC * TS / 128 / NW; ++i) {
        const int h = w + i * NW, slot = h * 64 + lane;
        const int row = slot / SPR, j = (slot % SPR) ^ qswz<KC>(row & 15);
        const int k = kc + 2 * j, r = min(row, rows - 1);
        dma16(k < k1 ? X + (long long)r * rs + k : zero, dst + h * 128);
      }
    } else {
#pragma unroll 1
      for (int i = 0; i < KC * TS / 32 / NW; ++i) {
        const int h = w + i * NW, d = h * 64 + lane, slot = d >> 2, e = d & 3;
        const int row = slot / SPR, j = (slot % SPR) ^ qswz<KC>(row & 15);
        const int k = kc + 2 * j + (e >> 1), r = min(row, rows - 1);
        const char *src = (const char *)(X + (long long)r * rs + (long long)k * ks) + (e & 1) * 4;
        dma4(k < k1 ? (const void *)src : (const void *)zero, dst + h * 32);
      }
    }
  }
}

// acc += sum over segments of alpha_s op(A_s) op(B_s)^T on a TS x TS tile,
// as run_product but staged with direct loads into two LDS buffers (separate
// arrays, so the compiler knows that loads into one never wait on reads of
// the other).  The loads of chunk c + 1 are issued before chunk c is
// multiplied and waited for after it.  Within a group of 8 k-values, MFMA
// step s of lane group g = lane / 16 takes k = 2g + s, which lets a Q row
// deliver both steps' values with one 16-byte read.  The alphas are applied
// to the accumulator: at a change of segment it is rescaled by
// alpha_old / alpha_new (segment weights are nonzero), and once at the end
// (an accumulator that starts from a tile, tk.init, starts at weight 1).
template <int KC, int WR, int WC, bool AQ, bool BQ, int TS, int S>
__device__ __forceinline__ void run_product_dma(const Task &tk, double *buf0, double *buf1,
                                                double *buf2, double *buf3,
                                                d4 (&acc)[TS / WR / 16][TS / WC / 16],
                                                int part = 0, int nparts = 1) {
  static_assert(S == 2 || S == 4, "two or four LDS stages");
  constexpr int NW = WR * WC;
  constexpr int LD = pld<TS>();
  constexpr int MR = TS / WR / 16, MC = TS / WC / 16;
  constexpr int OPS = KC * LD;    // doubles of one operand's panel (P is the larger layout)
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = w / WC, wc = w % WC;
  const int n0 = (tk.nseg > 0 && tk.seg[0].k1 > tk.seg[0].k0) ? (tk.seg[0].k1 - tk.seg[0].k0 + KC - 1) / KC : 0;
  const int n1 = (tk.nseg > 1 && tk.seg[1].k1 > tk.seg[1].k0) ? (tk.seg[1].k1 - tk.seg[1].k0 + KC - 1) / KC : 0;
  const int n2 = (tk.nseg > 2 && tk.seg[2].k1 > tk.seg[2].k0) ? (tk.seg[2].k1 - tk.seg[2].k0 + KC - 1) / KC : 0;
  const int all = n0 + n1 + n2;
  const int cb = (int)((long long)all * part / nparts), ce = (int)((long long)all * (part + 1) / nparts);
  if (ce <= cb) return;
  // per-lane LDS offsets (doubles): P reads at k = 2g (+ 8i + s), Q reads of slot 4i + g
  const int g = lane >> 4, r16 = lane & 15;
  const int pa = 2 * g * LD + wr * (TS / WR) + r16, pb = 2 * g * LD + wc * (TS / WC) + r16;
  int qo[KC / 8];
#pragma unroll
  for (int i = 0; i < KC / 8; ++i) qo[i] = r16 * KC + (((4 * i + g) ^ qswz<KC>(r16)) << 1);
  const int qa = wr * (TS / WR) * KC, qb = wc * (TS / WC) * KC;
  // chunk c: issue its loads into dst
  auto issue = [&](int c, double *dst) {
    const bool s1 = c >= n0, s2 = c >= n0 + n1;
    const double *A = pick3(s1, s2, tk.seg[0].A, tk.seg[1].A, tk.seg[2].A);
    const double *B = pick3(s1, s2, tk.seg[0].B, tk.seg[1].B, tk.seg[2].B);
    const int ars = pick3(s1, s2, tk.seg[0].ars, tk.seg[1].ars, tk.seg[2].ars);
    const int aks = pick3(s1, s2, tk.seg[0].aks, tk.seg[1].aks, tk.seg[2].aks);
    const int brs = pick3(s1, s2, tk.seg[0].brs, tk.seg[1].brs, tk.seg[2].brs);
    const int bks = pick3(s1, s2, tk.seg[0].bks, tk.seg[1].bks, tk.seg[2].bks);
    const int k0 = pick3(s1, s2, tk.seg[0].k0, tk.seg[1].k0, tk.seg[2].k0);
    const int k1 = pick3(s1, s2, tk.seg[0].k1, tk.seg[1].k1, tk.seg[2].k1);
    const int kc = k0 + (c - (s2 ? n0 + n1 : (s1 ? n0 : 0))) * KC;
    dma_operand<KC, NW, AQ, TS>(A, ars, aks, tk.m, kc, k1, dst, w, lane);
    dma_operand<KC, NW, BQ, TS>(B, brs, bks, tk.n, kc, k1, dst + OPS, w, lane);
  };
  auto seg_alpha = [&](int c) {
    const bool s1 = c >= n0, s2 = c >= n0 + n1;
    return pick3(s1, s2, tk.seg[0].alpha, tk.seg[1].alpha, tk.seg[2].alpha);
  };
  auto mma = [&](const double (&a0)[MR], const double (&a1)[MR], const double (&b0)[MC],
                 const double (&b1)[MC]) {
#pragma unroll
    for (int mi = 0; mi < MR; ++mi)
#pragma unroll
      for (int nj = 0; nj < MC; ++nj)
        acc[mi][nj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[mi], b0[nj], acc[mi][nj], 0, 0, 0);
#pragma unroll
    for (int mi = 0; mi < MR; ++mi)
#pragma unroll
      for (int nj = 0; nj < MC; ++nj)
        acc[mi][nj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[mi], b1[nj], acc[mi][nj], 0, 0, 0);
  };
  typedef double d2 __attribute__((ext_vector_type(2)));
  // one chunk (layouts AQ / BQ: operand in layout Q)
  auto compute = [&](const double *buf) {
    const double *As = buf, *Bs = buf + OPS;
#pragma unroll
    for (int i = 0; i < KC / 8; ++i) {
      double a0[MR], a1[MR], b0[MC], b1[MC];
#pragma unroll
      for (int x = 0; x < MR; ++x) {
        if constexpr (AQ) {
          const d2 v = *(const d2 *)(As + qa + x * 16 * KC + qo[i]);
          a0[x] = v.x; a1[x] = v.y;
        } else {
          a0[x] = As[pa + 8 * i * LD + x * 16];
          a1[x] = As[pa + (8 * i + 1) * LD + x * 16];
        }
      }
#pragma unroll
      for (int x = 0; x < MC; ++x) {
        if constexpr (BQ) {
          const d2 v = *(const d2 *)(Bs + qb + x * 16 * KC + qo[i]);
          b0[x] = v.x; b1[x] = v.y;
        } else {
          b0[x] = Bs[pb + 8 * i * LD + x * 16];
          b1[x] = Bs[pb + (8 * i + 1) * LD + x * 16];
        }
      }
      mma(a0, a1, b0, b1);
    }
  };
  double cur = seg_alpha(cb);
  if (tk.init && part == 0 && cur != 1.0) {
    // the incoming sum (a tile formed earlier) carries weight 1
    const double f = 1.0 / cur;
#pragma unroll
    for (int mi = 0; mi < MR; ++mi)
#pragma unroll
      for (int nj = 0; nj < MC; ++nj) acc[mi][nj] *= f;
  }
  auto rescale = [&](int c) {
    const double al = seg_alpha(c);
    if (al != cur) {
      const double f = cur / al;
#pragma unroll
      for (int mi = 0; mi < MR; ++mi)
#pragma unroll
        for (int nj = 0; nj < MC; ++nj) acc[mi][nj] *= f;
      cur = al;
    }
  };
  constexpr unsigned kVmcnt0 = 0x0F70;   // s_waitcnt vmcnt(0), other counters free
  if constexpr (S == 4) {
    // Chunk c sits in stage (c - cb) mod 4; the loads of c + 3 are issued once
    // every wave is past chunk c - 1 (the barrier), into that chunk's stage.
    // Before chunk c its own loads must be in: every chunk issues at least
    // kMin loads per wave and loads retire in order, so waiting until at most
    // kMin * (chunks issued after c) are outstanding is enough.
    constexpr int CPI = 128 / TS;
    constexpr int kMin = 2 * ((KC / CPI / NW) < (KC * TS / 128 / NW) ? (KC / CPI / NW)
                                                                       : (KC * TS / 128 / NW));
    static_assert(kMin >= 1 && 2 * kMin < 64, "vmcnt range");
    // The barrier is s_barrier alone: __syncthreads() would also fence memory
    // and so wait for every load in flight.  This wave's LDS reads of the
    // stage about to be refilled are waited for (lgkmcnt(0)) with the loads.
    constexpr unsigned kLgkm0 = 0x0070;   // lgkmcnt(0) and vmcnt(0); OR in vmcnt
    auto wait_for = [&](int cc) {
      const int after = min(2, ce - 1 - cc);
      if (after >= 2) __builtin_amdgcn_s_waitcnt(kLgkm0 | (2 * kMin));
      else if (after == 1) __builtin_amdgcn_s_waitcnt(kLgkm0 | kMin);
      else __builtin_amdgcn_s_waitcnt(kLgkm0);
    };
    auto step = [&](int cc, double *now, double *next) {
      wait_for(cc);
      __builtin_amdgcn_s_barrier();
      if (cc + 3 < ce) issue(cc + 3, next);
      __builtin_amdgcn_sched_barrier(0);
      rescale(cc);
      compute(now);
    };
    issue(cb, buf0);
    if (cb + 1 < ce) issue(cb + 1, buf1);
    if (cb + 2 < ce) issue(cb + 2, buf2);
    for (int c = cb; c < ce; c += 4) {
      step(c, buf0, buf3);
      if (c + 1 >= ce) break;
      step(c + 1, buf1, buf0);
      if (c + 2 >= ce) break;
      step(c + 2, buf2, buf1);
      if (c + 3 >= ce) break;
      step(c + 3, buf3, buf2);
    }
    __syncthreads();
#pragma unroll
    for (int mi = 0; mi < MR; ++mi)
#pragma unroll
      for (int nj = 0; nj < MC; ++nj) acc[mi][nj] *= cur;
    return;
  }
  issue(cb, buf0);
  __builtin_amdgcn_s_waitcnt(kVmcnt0);
  __syncthreads();
  for (int c = cb; c < ce; c += 2) {
    if (c + 1 < ce) issue(c + 1, buf1);
    __builtin_amdgcn_sched_barrier(0);
    rescale(c);
    compute(buf0);
    __builtin_amdgcn_s_waitcnt(kVmcnt0);
    __syncthreads();
    if (c + 1 >= ce) break;
    if (c + 2 < ce) issue(c + 2, buf0);
    __builtin_amdgcn_sched_barrier(0);
    rescale(c + 1);
    compute(buf1);
    __builtin_amdgcn_s_waitcnt(kVmcnt0);
    __syncthreads();
  }
#pragma unroll
  for (int mi = 0; mi < MR; ++mi)
#pragma unroll
    for (int nj = 0; nj < MC; ++nj) acc[mi][nj] *= cur;
}

// Output mapping of v_mfma_f64_16x16x4f64: lane l, element r -> row (l>>4) + 4r, col l&15.
__device__ inline int acc_row(int wr, int mi, int lane, int r) {
  return wr * 32 + mi * 16 + (lane >> 4) + 4 * r;
}
__device__ inline int acc_col(int wc, int nj, int lane) { return wc * 32 + nj * 16 + (lane & 15); }

// Every lane takes the value of lane J of its own row of 16 lanes (DPP
// row_newbcast, one 64-bit move; every lane is written, so the value the move
// would keep in unwritten lanes is immaterial); row_bcast selects J from a
// value that is a constant once the caller's loop is unrolled.
template <int J>
__device__ __forceinline__ double row_bcast_c(double x) {
  return __builtin_amdgcn_update_dpp(x, x, 0x150 + J, 0xf, 0xf, true);
}
__device__ __forceinline__ double row_bcast(double x, int j) {
  switch (j) {
    case 0: return row_bcast_c<0>(x);
    case 1: return row_bcast_c<1>(x);
    case 2: return row_bcast_c<2>(x);
    case 3: return row_bcast_c<3>(x);
    case 4: return row_bcast_c<4>(x);
    case 5: return row_bcast_c<5>(x);
    case 6: return row_bcast_c<6>(x);
    case 7: return row_bcast_c<7>(x);
    case 8: return row_bcast_c<8>(x);
    case 9: return row_bcast_c<9>(x);
    case 10: return row_bcast_c<10>(x);
    case 11: return row_bcast_c<11>(x);
    case 12: return row_bcast_c<12>(x);
    case 13: return row_bcast_c<13>(x);
    case 14: return row_bcast_c<14>(x);
    default: return row_bcast_c<15>(x);
  }
}

// 1/sqrt(x) from the hardware estimate refined by two Newton steps
// (y <- y + y(1 - x y^2)/2), which take it to full double precision for the
// positive pivots of a Cholesky factorization.
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
  y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
  return y;
}

// One 16 x 16 block of X = L^{-1} below the diagonal, by one wave:
// X_ij = -X_ii sum_{m=j}^{i-1} L_im X_mj (L in A, X in X, both row-major with
// ld TLD); P is the wave's own 16 x 16 scratch (ld TLD) for the sum.
__device__ __forceinline__ void inv_block(const double *A, double *X, double *P, int i, int j) {
  const int lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
  d4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int m = j; m < i; ++m) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double av = A[(16 * i + lr) * TLD + 16 * m + 4 * q + lk];
      const double bv = X[(16 * m + 4 * q + lk) * TLD + 16 * j + lr];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) P[(lk + 4 * r) * TLD + lr] = acc[r];
  // the wave reads back what its own lanes wrote (LDS operations of a wave
  // complete in order)
  __builtin_amdgcn_wave_barrier();
  d4 acc2 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double av = X[(16 * i + lr) * TLD + 16 * i + 4 * q + lk];
    const double bv = P[(4 * q + lk) * TLD + lr];
    acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc2, 0, 0, 0);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) X[(16 * i + lk + 4 * r) * TLD + 16 * j + lr] = -acc2[r];
}

// Cholesky + inverse of one 64 x 64 tile held in LDS (A, row-major, ld TLD;
// rows/cols >= w padded with the identity).  16 x 16 diagonal blocks are
// factored and inverted by one wave (rows in lanes, columns broadcast from
// lane to lane); the panel solves, trailing updates and the blocks of
// X = L^{-1} below the diagonal (X_ij = -X_ii sum_m L_im X_mj) run on the
// matrix cores, the row blocks of X on the other waves while wave 0 factors
// the next diagonal block.  Writes inv(L)
// (zeros above the diagonal) to Lout and sum log L_jj; a pivot that is not
// positive sets *info to its 1-based row (row_off + local row) if smaller.
// dlog holds the 64 diagonal entries of L (its 2 * kTile doubles leave room).
// If Mout is set, M = X^T X = inv(A) (64 x 64, column-major) is written there too.
__device__ void chol_inv_tile(double *A, double *X, double *dlog, int w, double *Lout,
                              long long ldl, double *ldsum, int row_off, int *info, double *Mout) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nb = (w + 15) / 16;
  const int lr = lane & 15, lk = lane >> 4;
  for (int k = 0; k < nb; ++k) {
    // (a) factor and invert the diagonal block (k,k) in wave 0.  Cholesky,
    //     right-looking: lane i holds row i (every row of 16 lanes holds the
    //     same copy); at pivot j column j (= row j of the symmetric trailing
    //     block) reaches every lane by row broadcasts, so the only latency
    //     between pivots is the pivot's reciprocal and one update.  Row j of
    //     X = L^{-1} (lane c: column c) follows in the same pivot, by forward
    //     substitution with row j of L, final on lane j once pivot j is done.
    if (wv == 0) {
      const int r0 = 16 * k;
      double a[16], x[16];
      // Lane i computes row i of the factor; its entries above the diagonal
      // are scratch (they only ever feed other entries above the diagonal),
      // so the updates run on every lane without per-column lane masks.
      const int lr16 = lane & 15;
#pragma unroll
      for (int c = 0; c < 16; ++c) a[c] = A[(r0 + lr16) * TLD + r0 + c];
      double dg = 1.0;   // lane j keeps L_jj
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        double cv[16];
#pragma unroll
        for (int m = j; m < 16; ++m) cv[m] = row_bcast(a[j], m);
        const double piv = cv[j];
        const double rs = rsqrt_nr(piv);
        const double ip = rs * rs;   // 1/piv within a few ulp, without a second Newton chain
        // L_jj = piv / sqrt(piv), the same value on every lane
        dg = (lr16 == j) ? piv * rs : dg;
        // A_im -= L_ij L_mj = A_ij A_mj / piv for m > j; then L_ij = A_ij / sqrt(piv)
        const double wj = a[j] * ip;
#pragma unroll
        for (int m = j + 1; m < 16; ++m) a[m] = fma(-wj, cv[m], a[m]);
        a[j] *= rs;
        // X_jc = (delta_jc - sum_{m<j} L_jm X_mc) / L_jj; entries above the
        // diagonal come out zero because the right-hand side is e_c
        double s0 = (j == lane) ? 1.0 : 0.0, s1 = 0.0;
#pragma unroll
        for (int m = 0; m < j; ++m) {
          const double l = row_bcast(a[m], j);
          if (m & 1) s1 = fma(-l, x[m], s1);
          else s0 = fma(-l, x[m], s0);
        }
        x[j] = (s0 + s1) * rs;
      }
      if (lane < 16) {
#pragma unroll
        for (int c = 0; c < 16; ++c) A[(r0 + lane) * TLD + r0 + c] = a[c];
#pragma unroll
        for (int i = 0; i < 16; ++i) X[(r0 + i) * TLD + r0 + lane] = x[i];
        dlog[r0 + lane] = dg;   // logs taken once, at the end
      }
      // L_jj is NaN exactly when the pivot is not positive (or not a
      // number): the first such row is the failure
      const bool ok = (dg > 0.0) || lane >= 16 || r0 + lane >= w;
      const unsigned long long badm = __ballot(!ok);
      if (badm && lane == 0) atomicMin(info, row_off + r0 + __ffsll(badm));
    } else if (wv < k) {
      // row block k-1 of X (block j = wv-1 < k-1): L_{k-1,m} (m < k-1), the
      // rows of X above and X_{k-1,k-1} are final; the scratch is the unused
      // block (0, wv) above the diagonal
      inv_block(A, X, A + 16 * wv, k - 1, wv - 1);
    }
    __syncthreads();
    if (k + 1 >= nb) break;
    // (b) panel blocks L_ik = A_ik Linv_kk^T, i > k
    {
      const int i = k + 1 + wv;
      if (i < nb) {
        d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double av = A[(16 * i + lr) * TLD + 16 * k + 4 * q + lk];
          const double bv = X[(16 * k + lr) * TLD + 16 * k + 4 * q + lk];
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) A[(16 * i + lk + 4 * r) * TLD + 16 * k + lr] = acc[r];
      }
    }
    __syncthreads();
    // (c) trailing blocks A_ij -= L_ik L_jk^T, k < j <= i < nb
    {
      const int nrem = nb - 1 - k;
      const int nblk = nrem * (nrem + 1) / 2;
      for (int e = wv; e < nblk; e += 4) {
        int ii, jj;
        tri_decode(e, ii, jj);
        const int i = k + 1 + ii, j = k + 1 + jj;
        d4 acc;
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] = A[(16 * i + lk + 4 * r) * TLD + 16 * j + lr];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double av = A[(16 * i + lr) * TLD + 16 * k + 4 * q + lk];
          const double bv = A[(16 * j + lr) * TLD + 16 * k + 4 * q + lk];
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-av, bv, acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) A[(16 * i + lk + 4 * r) * TLD + 16 * j + lr] = acc[r];
      }
    }
    __syncthreads();
  }
  // the last row block of X (blocks j < nb-1 on waves j; scratch above the
  // diagonal of block row 0) and, on wave 3, the sum of log L_jj
  if (wv < nb - 1) {
    inv_block(A, X, A + 16 * (wv + 1), nb - 1, wv);
  } else if (wv == 3) {
    double v = (lane < w) ? log(dlog[lane]) : 0.0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) *ldsum = v;
  }
  __syncthreads();
  {
    // inv(L) (zeros above the diagonal) to Lout: every read is issued before the stores
    double v[kTile * kTile / kThreads];
#pragma unroll
    for (int q = 0; q < kTile * kTile / kThreads; ++q) {
      const int e = tid + q * kThreads;
      const int r = e & (kTile - 1), c = e / kTile;
      v[q] = (c <= r) ? X[r * TLD + c] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < kTile * kTile / kThreads; ++q) {
      const int e = tid + q * kThreads;
      const int r = e & (kTile - 1), c = e / kTile;
      if (r < w && c < w) gst(Lout + r + (long long)c * ldl, v[q]);
    }
  }
  if (Mout) {
    // M = X^T X = inv(A) is symmetric and M_rc = sum_{k >= max(r,c)} X_kr X_kc
    // (X lower triangular), so of the 32 x 32 blocks only (0,0), (1,0) and
    // (1,1) are computed, each wave over 32 values of k: wave 0 takes block
    // (0,0) over k < 32 and wave 1 over k >= 32 (its sum reaches wave 0 through
    // LDS), waves 2 and 3 take blocks (1,0) and (1,1), where only k >= 32
    // contributes.  Block (0,1) is stored as the transpose of block (1,0).
    // Only the lower triangle of X in LDS is defined: entries above it are read as 0.
    const int br = wv >> 1, bc = (wv == 3) ? 1 : 0;
    const int k0 = (wv == 0) ? 0 : 32;
    d4 mac[2][2];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int nj = 0; nj < 2; ++nj) mac[mi][nj] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < 32; kk += 4) {
      const int kq = k0 + kk + lk;
      double av[2], bv[2];
#pragma unroll
      for (int mi = 0; mi < 2; ++mi) {
        const int r = br * 32 + mi * 16 + lr;
        const double v = X[kq * TLD + r];
        av[mi] = (kq >= r) ? v : 0.0;
      }
#pragma unroll
      for (int nj = 0; nj < 2; ++nj) {
        const int c = bc * 32 + nj * 16 + lr;
        const double v = X[kq * TLD + c];
        bv[nj] = (kq >= c) ? v : 0.0;
      }
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < 2; ++nj)
          mac[mi][nj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[mi], bv[nj], mac[mi][nj], 0, 0, 0);
    }
    // the factor in A is no longer needed: wave 1's partial sums pass through it
    if (wv == 1) {
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < 2; ++nj)
#pragma unroll
          for (int r = 0; r < 4; ++r) A[(mi * 16 + lk + 4 * r) * TLD + nj * 16 + lr] = mac[mi][nj][r];
    }
    __syncthreads();
    if (wv != 1) {
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < 2; ++nj)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = br * 32 + mi * 16 + lk + 4 * r, col = bc * 32 + nj * 16 + lr;
            double v = mac[mi][nj][r];
            if (wv == 0) v += A[(mi * 16 + lk + 4 * r) * TLD + nj * 16 + lr];
            gst(Mout + row + (long long)col * kTile, v);
            if (wv == 2) gst(Mout + col + (long long)row * kTile, v);
          }
    }
  }
}

// TK_LCHAIN on a 64 x 64 tile: acc = -A1 (A0 B0), A1 (tk.m x tk.m, lower, from
// global memory) multiplying the intermediate T = A0 B0 (tk.m x 64) from the left.
template <int KC, bool SHORT>
__device__ __forceinline__ void left_chain_product(const Task &tk, double *smem, d4 (&acc)[2][2]) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w >> 1, wc = w & 1;
  Task t1 = tk;
  t1.nseg = 1;
  run_product<KC, kTile, 2, 2, 2, SHORT>(t1, smem, acc);   // rows >= tk.m come out zero
  if (tk.src) {
    // plus the tile at src (ld = ldc): the running sum of the earlier terms
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int nj = 0; nj < 2; ++nj)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = acc_row(wr, mi, lane, r), col = acc_col(wc, nj, lane);
          const double v = gld(tk.src + min(row, tk.m - 1) + (long long)min(col, tk.n - 1) * tk.ldc);
          if (row < tk.m && col < tk.n) acc[mi][nj][r] += v;
        }
  }
  double *TA = smem, *TB = smem + kTile * TLD;
  // T[k][c] -> TB[c][k]
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int nj = 0; nj < 2; ++nj)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        TB[acc_col(wc, nj, lane) * TLD + acc_row(wr, mi, lane, r)] = acc[mi][nj][r];
  const double *A1 = tk.seg[1].A;
  const long long aks = tk.seg[1].aks;
  const int w1 = tk.m;
#pragma unroll
  for (int q = 0; q < kTile * kTile / kThreads; ++q) {
    const int e = tid + q * kThreads;
    const int r = e & (kTile - 1), k = e / kTile;
    const double v = gld(A1 + min(r, w1 - 1) + (long long)min(k, w1 - 1) * aks);
    TA[r * TLD + k] = (r < w1 && k < w1) ? v : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int nj = 0; nj < 2; ++nj) acc[mi][nj] = d4{0.0, 0.0, 0.0, 0.0};
  for (int kk = 0; kk < kTile; kk += 4) {
    const int kq = kk + (lane >> 4);
    double av[2], bv[2];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi) av[mi] = TA[(wr * 32 + mi * 16 + (lane & 15)) * TLD + kq];
#pragma unroll
    for (int nj = 0; nj < 2; ++nj) bv[nj] = TB[(wc * 32 + nj * 16 + (lane & 15)) * TLD + kq];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int nj = 0; nj < 2; ++nj)
        acc[mi][nj] = __builtin_amdgcn_mfma_f64_16x16x4f64(-av[mi], bv[nj], acc[mi][nj], 0, 0, 0);
  }
  __syncthreads();
}

// TK_CHAIN on a 64 x 64 tile: acc = -T0 T1^T (+ seg[2]).  T0 = A0 B0^T (tk.m x 64,
// k = 64) comes from the regular product loop.  T1 is A1 itself (seg[1].B null),
// or, in the Cholesky-capable kernel (FATK), A1 B1^T formed here as well when
// seg[1].B is set (T1 = T0 when A1 = A0).  Both are staged in LDS (row-major,
// ld TLD) for the second product (k = 64).  When T1 = T0 the region of T1 is
// free: stage_c(region) may put the caller's C there before the barrier ahead
// of the second product; returns whether it did.
template <int KC, bool FATK, class StageC>
__device__ __forceinline__ bool chain_product(const Task &tk, double *smem, d4 (&acc)[2][2],
                                              StageC stage_c) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w >> 1, wc = w & 1;
  const bool formed = FATK && tk.seg[1].B != nullptr;
  const bool same = formed && tk.seg[1].A == tk.seg[0].A;
  // A1 itself: the Cholesky-capable kernel loads it first, so that its
  // latency overlaps the first product's loads (it holds 32 more registers)
  const double *A1 = tk.seg[1].A;
  const long long aks = tk.seg[1].aks;
  double b1[kTile * kTile / kThreads];
  auto load_b1 = [&]() {
#pragma unroll
    for (int q = 0; q < kTile * kTile / kThreads; ++q) {
      const int e = tid + q * kThreads;
      const int c = e & (kTile - 1), k = e / kTile;
      b1[q] = gld(A1 + min(c, tk.n - 1) + (long long)k * aks);
    }
  };
  if (FATK && !formed) load_b1();
  Task t1 = tk;
  t1.n = kTile;
  t1.nseg = 1;
  run_product<KC, kTile, 2, 2, 2, FATK>(t1, smem, acc);   // ends with a barrier
  double *TA = smem, *TB = smem + kTile * TLD;
  auto stage = [&](double *T, const d4 (&v)[2][2]) {
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int nj = 0; nj < 2; ++nj)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          T[acc_row(wr, mi, lane, r) * TLD + acc_col(wc, nj, lane)] = v[mi][nj][r];
  };
  bool c_staged = false;
  if (formed && !same) {
    d4 t0[2][2];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int nj = 0; nj < 2; ++nj) {
        t0[mi][nj] = acc[mi][nj];
        acc[mi][nj] = d4{0.0, 0.0, 0.0, 0.0};
      }
    Task t2 = tk;
    t2.seg[0] = tk.seg[1];
    t2.seg[0].alpha = 1.0;
    t2.m = tk.n;
    t2.n = kTile;
    t2.nseg = 1;
    run_product<KC, kTile, 2, 2, 2, FATK>(t2, smem, acc);   // ends with a barrier
    stage(TA, t0);
    stage(TB, acc);
  } else {
    stage(TA, acc);
    if (formed) {
      TB = TA;
      c_staged = stage_c(smem + kTile * TLD);
    } else {
      if (!FATK) load_b1();
#pragma unroll
      for (int q = 0; q < kTile * kTile / kThreads; ++q) {
        const int e = tid + q * kThreads;
        const int c = e & (kTile - 1), k = e / kTile;
        TB[c * TLD + k] = b1[q];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int nj = 0; nj < 2; ++nj) acc[mi][nj] = d4{0.0, 0.0, 0.0, 0.0};
  for (int kk = 0; kk < kTile; kk += 4) {
    const int kq = kk + (lane >> 4);
    double av[2], bv[2];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi) av[mi] = TA[(wr * 32 + mi * 16 + (lane & 15)) * TLD + kq];
#pragma unroll
    for (int nj = 0; nj < 2; ++nj) bv[nj] = TB[(wc * 32 + nj * 16 + (lane & 15)) * TLD + kq];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int nj = 0; nj < 2; ++nj)
        acc[mi][nj] = __builtin_amdgcn_mfma_f64_16x16x4f64(-av[mi], bv[nj], acc[mi][nj], 0, 0, 0);
  }
  __syncthreads();
  if (tk.seg[2].k1 > tk.seg[2].k0) {   // a further plain product term
    Task t3 = tk;
    t3.seg[0] = tk.seg[2];
    t3.nseg = 1;
    run_product<KC, kTile, 2, 2, 2, FATK>(t3, smem, acc);
  }
  return c_staged;
}

// Owner of workgroup task q in a launch over n_items items whose task counts
// are count(item): the lanes of each wave evaluate 64 items at a time, an
// inclusive prefix sum over the wave finds the item, and q becomes the index of
// the task within it.  Returns n_items when q is past the last task.
template <class Count>
__device__ __forceinline__ int find_item(const ItemDev *items, int n_items, int &q, Count count) {
  const int lane = threadIdx.x & 63;
  int base = 0;
  for (int i0 = 0; i0 < n_items; i0 += 64) {
    const int i = i0 + lane;
    const int c = (i < n_items) ? count(items[i]) : 0;
    int incl = c;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int v = __shfl_up(incl, off);
      incl += (lane >= off) ? v : 0;
    }
    const int tot = __builtin_amdgcn_readfirstlane(__shfl(incl, 63));
    if (q < base + tot) {
      const unsigned long long m = __ballot(base + incl > q);
      const int l = __ffsll((unsigned long long)m) - 1;
      // the results are wave-uniform; say so, so that the item's fields are
      // read with scalar loads
      q = __builtin_amdgcn_readfirstlane(q - base - __shfl(incl - c, l));
      return __builtin_amdgcn_readfirstlane(i0 + l);
    }
    base += tot;
  }
  q -= base;   // past the last task: q counts on from the end
  return n_items;
}

// One launch covers the tasks of `phase` and, if phase2 >= 0, of `phase2` as
// well (two independent phases of the same step), item by item.
template <bool FAT>
__global__ __launch_bounds__(kThreads, FAT ? 1 : 2) void tile_phase_kernel(const ItemDev *__restrict__ items,
                                                              int n_items, int phase, int phase2,
                                                              int t, int p) {
  __shared__ double smem[FAT ? kFatLds : kLeanLds];
  int q = blockIdx.x;
  int ii;
  int ph = phase;
  if ((phase == PH_STEP || phase == PH_STEPF) && phase2 < 0) {
    // a Cholesky step: the long tasks of every item take the first
    // workgroups, so that none of them waits for a second round behind short ones
    ii = find_item(items, n_items, q, [&](const ItemDev &x) {
      return step_split(x.nP, phase, t, p, x.nrun).nlong();
    });
    const bool is_long = ii < n_items;
    if (!is_long)
      ii = find_item(items, n_items, q, [&](const ItemDev &x) {
        return step_split(x.nP, phase, t, p, x.nrun).nshort();
      });
    if (ii >= n_items) return;
    q = step_task_local(step_split(items[ii].nP, phase, t, p, items[ii].nrun), is_long, q);
  } else {
    // tasks are ordered item by item, the item's `phase` tasks before its `phase2` ones
    ii = find_item(items, n_items, q, [&](const ItemDev &x) {
      return phase_tasks(x, phase, t, p) + (phase2 >= 0 ? phase_tasks(x, phase2, t, p) : 0);
    });
    if (ii >= n_items) return;
    const int c1 = phase_tasks(items[ii], phase, t, p);
    if (q >= c1) {
      q -= c1;
      ph = phase2;
    }
  }
  const ItemDev it = items[ii];
  Task tk;
  decode<FAT ? kFatOnly : kLeanOnly>(it, ph, t, p, q, tk);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w >> 1, wc = w & 1;
  if (tk.kind == TK_NONE) return;
  if (tk.kind == TK_COPY || tk.kind == TK_ZERO) {
    // out-of-range lanes rewrite the clamped edge element with its own value
    double v[kTile * kTile / kThreads];
#pragma unroll
    for (int q = 0; q < kTile * kTile / kThreads; ++q) {
      const int e = tid + q * kThreads;
      const int r = min(e & (kTile - 1), tk.m - 1), c = min(e / kTile, tk.n - 1);
      v[q] = (tk.kind == TK_COPY) ? gld(tk.src + r + c * tk.ldc) : 0.0;
    }
#pragma unroll
    for (int q = 0; q < kTile * kTile / kThreads; ++q) {
      const int e = tid + q * kThreads;
      const int r = min(e & (kTile - 1), tk.m - 1), c = min(e / kTile, tk.n - 1);
      gst(tk.C + r + c * tk.ldc, v[q]);
    }
    return;
  }
  d4 acc[2][2];
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int nj = 0; nj < 2; ++nj) acc[mi][nj] = d4{0.0, 0.0, 0.0, 0.0};
  if (tk.kind == TK_PRODUCT && tk.init) {
    // the sum starts from a tile formed earlier
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int nj = 0; nj < 2; ++nj)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = min(acc_row(wr, mi, lane, r), tk.m - 1);
          const int col = min(acc_col(wc, nj, lane), tk.n - 1);
          acc[mi][nj][r] = gld(tk.init + row + (long long)col * tk.ldc);
        }
  }
  constexpr int KC = FAT ? kFatKC : kLeanKC;
  // C of the tile that is factored here is loaded (column by column, in
  // full lines) before the products start, so that its latency overlaps theirs
  constexpr int kPer = kTile * kTile / kThreads;
  double cpre[FAT ? kPer : 1];
  if constexpr (FAT) {
    if (tk.chol) {
#pragma unroll
      for (int q = 0; q < kPer; ++q) {
        const int e = tid + q * kThreads;
        const int r = min(e & (kTile - 1), tk.m - 1), c = min(e / kTile, tk.n - 1);
        cpre[q] = gld(tk.C + r + c * tk.ldc);
      }
    }
  }
  // the factored tile's beta C, identity-padded, in the layout of the tile in LDS
  auto c_fill = [&](double *Tc) -> bool {
    if constexpr (FAT) {
      if (!tk.chol) return false;
#pragma unroll
      for (int q = 0; q < kPer; ++q) {
        const int e = tid + q * kThreads;
        const int r = e & (kTile - 1), c = e / kTile;
        Tc[r * TLD + c] = (r < tk.m && c < tk.n) ? tk.beta * cpre[q] : ((r == c) ? 1.0 : 0.0);
      }
      return true;
    } else {
      (void)Tc;
      return false;
    }
  };
  bool c_staged = false;
  if (tk.kind == TK_CHAIN) c_staged = chain_product<KC, FAT>(tk, smem, acc, c_fill);
  else if (tk.kind == TK_LCHAIN) left_chain_product<KC, FAT>(tk, smem, acc);
  else run_product<KC, kTile, 2, 2, 2, FAT>(tk, smem, acc);

  if constexpr (FAT) {
    if (tk.chol) {
      double *A = smem;
      double *X = smem + kTile * TLD;
      double *dlog = smem + 2 * kTile * TLD;
      // beta C (identity padding beyond the tile) in LDS, then each lane adds
      // its part of the product.  A chained task staged C in the region of X
      // already (ahead of its second product): one pass from there into A.
      if (c_staged) {
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
#pragma unroll
          for (int nj = 0; nj < 2; ++nj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int row = acc_row(wr, mi, lane, r), col = acc_col(wc, nj, lane);
              const double v = X[row * TLD + col];
              A[row * TLD + col] = (row < tk.m && col < tk.n) ? v + acc[mi][nj][r] : v;
            }
      } else {
        c_fill(A);
        __syncthreads();
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
#pragma unroll
          for (int nj = 0; nj < 2; ++nj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int row = acc_row(wr, mi, lane, r), col = acc_col(wc, nj, lane);
              if (row < tk.m && col < tk.n) A[row * TLD + col] += acc[mi][nj][r];
            }
      }
      __syncthreads();
      chol_inv_tile(A, X, dlog, tk.m, tk.Lout, tk.ldl, tk.ldsum, tk.row_off, it.info, tk.Mout);
      return;
    }
  }
  // plain (and mirrored) store; C is read first (clamped, unconditional) when beta != 0
  double cold[2][2][4];
  if (tk.beta != 0.0) {
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int nj = 0; nj < 2; ++nj)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = min(acc_row(wr, mi, lane, r), tk.m - 1);
          const int col = min(acc_col(wc, nj, lane), tk.n - 1);
          cold[mi][nj][r] = tk.beta * gld(tk.C + row + col * tk.ldc);
        }
  } else {
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int nj = 0; nj < 2; ++nj)
#pragma unroll
        for (int r = 0; r < 4; ++r) cold[mi][nj][r] = 0.0;
  }
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int nj = 0; nj < 2; ++nj)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[mi][nj][r] += cold[mi][nj][r];
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int nj = 0; nj < 2; ++nj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = acc_row(wr, mi, lane, r), col = acc_col(wc, nj, lane);
        if (row < tk.m && col < tk.n) {
          const double v = acc[mi][nj][r];
          double *cp = tk.C + row + col * tk.ldc;
          if (tk.mirror && tk.diagtile) {
            if (row >= col) {
              gst(cp, v);
              gst(tk.Cm + col + row * tk.ldc, v);
            }
          } else {
            gst(cp, v);
            if (tk.mirror) gst(tk.Cm + col + row * tk.ldc, tk.mirror == 2 ? 0.0 : v);
          }
        }
      }
}

// Output tiles of the b x b products (TS x TS): WR x WC waves, each owning a
// block of (TS / WR) x (TS / WC) outputs in 16 x 16 MFMA blocks.
// The dispatcher deals workgroups round-robin to the 8 XCDs (workgroup id
// mod 8), each with its own L2.  Renumbering so that XCD x receives one
// contiguous range of tiles keeps tiles that share operand panels on one L2
// and gives every XCD the same mix of short and long tiles.
__device__ __forceinline__ int xcd_contiguous(int bid, int n) {
  const int x = bid & 7, j = bid >> 3;
  const int per = n >> 3, rem = n & 7;
  return x * per + min(x, rem) + j;
}

// With ks > 1 the k range of every tile is split over ks workgroups (adjacent
// task numbers, so on one XCD); part h writes its partial product, without
// beta or mirroring, to it.P + h*b*b at the tile's position (ld b), and
// splitk_reduce_kernel forms C.
// With phase2 >= 0 (and ks = 1) the launch also runs the nside tasks of the
// independent side phase phase2 of the same step (64-tile form: products of
// the arrow rows and tile copies): they take the first workgroups, so they
// start at once and spread over the XCDs, and the product tiles follow (their
// count rounded up to a multiple of 8 so that the XCD of a workgroup is still
// its number mod 8).
// LAY (layouts staged by direct loads): bit 0 A in layout Q, bit 1 B in layout Q.
template <int V, int LAY = 0>
__global__ __launch_bounds__(big_threads<V>(), BigCfg<V>::OCC) void tile_product_kernel(
    const ItemDev *__restrict__ items, int n_items, int phase, int phase2, int nside, int t,
    int ks) {
  using C = BigCfg<V>;
  constexpr int TS = C::TS;
  constexpr int MR = TS / C::WR / 16, MC = TS / C::WC / 16;
  const int nsp = (nside + 7) & ~7;
  const bool side = (int)blockIdx.x < nsp;
  int q, part = 0;
  if (side) {
    if ((int)blockIdx.x >= nside) return;
    q = blockIdx.x;
  } else {
    const int qa = xcd_contiguous(blockIdx.x - nsp, gridDim.x - nsp);
    q = qa / ks;
    part = qa - q * ks;
  }
  const int ii =
      side ? find_item(items, n_items, q, [&](const ItemDev &x) { return phase_tasks(x, phase2, t, 0); })
           : find_item(items, n_items, q,
                       [&](const ItemDev &x) { return phase_tasks(x, phase, t, 0, TS == kBig); });
  if (ii >= n_items) return;
  const ItemDev it = items[ii];
  Task tk;
  // LAY names the phases of a direct-load launch (big_layouts); the
  // register-staged layouts run every phase
  constexpr int kOnly = C::DMA ? LAY : -1;
  if (side) decode<kOnly>(it, phase2, t, 0, q, tk);
  else decode_big<TS, kOnly>(it, phase, t, q, tk);
  if (tk.kind == TK_COPY) {
    for (int e = threadIdx.x; e < kTile * kTile; e += blockDim.x) {
      const int r = e & (kTile - 1), c = e / kTile;
      if (r < tk.m && c < tk.n) gst(tk.C + r + (long long)c * tk.ldc, gld(tk.src + r + (long long)c * tk.ldc));
    }
    return;
  }
  if (tk.kind != TK_PRODUCT) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w / C::WC, wc = w % C::WC;
  d4 acc[MR][MC];
#pragma unroll
  for (int mi = 0; mi < MR; ++mi)
#pragma unroll
    for (int nj = 0; nj < MC; ++nj) acc[mi][nj] = d4{0.0, 0.0, 0.0, 0.0};
  if (tk.init && part == 0) {
    // the sum starts from a tile formed earlier (the one split-k part adds it)
#pragma unroll
    for (int mi = 0; mi < MR; ++mi)
#pragma unroll
      for (int nj = 0; nj < MC; ++nj)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = min(wr * (TS / C::WR) + mi * 16 + (lane >> 4) + 4 * r, tk.m - 1);
          const int col = min(wc * (TS / C::WC) + nj * 16 + (lane & 15), tk.n - 1);
          acc[mi][nj][r] = gld(tk.init + row + (long long)col * tk.ldc);
        }
  }
  if constexpr (C::DMA && C::STAGES == 4) {
    __shared__ __attribute__((aligned(16))) double stage0[big_lds<V>() / 4];
    __shared__ __attribute__((aligned(16))) double stage1[big_lds<V>() / 4];
    __shared__ __attribute__((aligned(16))) double stage2[big_lds<V>() / 4];
    __shared__ __attribute__((aligned(16))) double stage3[big_lds<V>() / 4];
    run_product_dma<C::KC, C::WR, C::WC, (LAY & 1) != 0, (LAY & 2) != 0, TS, 4>(
        tk, stage0, stage1, stage2, stage3, acc, part, ks);
  } else if constexpr (C::DMA) {
    __shared__ __attribute__((aligned(16))) double stage0[big_lds<V>() / 2];
    __shared__ __attribute__((aligned(16))) double stage1[big_lds<V>() / 2];
    run_product_dma<C::KC, C::WR, C::WC, (LAY & 1) != 0, (LAY & 2) != 0, TS, 2>(
        tk, stage0, stage1, nullptr, nullptr, acc, part, ks);
  } else {
    __shared__ double smem[big_lds<V>()];
    static_assert(TS == kBig, "register-staged layouts are 128-wide");
    run_product<C::KC, kBig, C::WR, C::WC, C::DEPTH>(tk, smem, acc, part, ks);
  }
  if (ks > 1) {
    double *Pp = it.P + (long long)part * it.b * it.b + (long long)tk.ti * TS +
                 (long long)tk.tj * TS * it.b;
#pragma unroll
    for (int mi = 0; mi < MR; ++mi)
#pragma unroll
      for (int nj = 0; nj < MC; ++nj)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = wr * (TS / C::WR) + mi * 16 + (lane >> 4) + 4 * r;
          const int col = wc * (TS / C::WC) + nj * 16 + (lane & 15);
          if (row < tk.m && col < tk.n) gst(Pp + row + (long long)col * it.b, acc[mi][nj][r]);
        }
    return;
  }
#pragma unroll
  for (int mi = 0; mi < MR; ++mi)
#pragma unroll
    for (int nj = 0; nj < MC; ++nj) {
      double cold[4];
      if (tk.beta != 0.0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = min(wr * (TS / C::WR) + mi * 16 + (lane >> 4) + 4 * r, tk.m - 1);
          const int col = min(wc * (TS / C::WC) + nj * 16 + (lane & 15), tk.n - 1);
          cold[r] = gld(tk.C + row + col * tk.ldc);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[mi][nj][r] += tk.beta * cold[r];
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = wr * (TS / C::WR) + mi * 16 + (lane >> 4) + 4 * r;
        const int col = wc * (TS / C::WC) + nj * 16 + (lane & 15);
        if (row < tk.m && col < tk.n) {
          const double v = acc[mi][nj][r];
          double *cp = tk.C + row + col * tk.ldc;
          if (tk.mirror && tk.diagtile) {
            if (row >= col) {
              gst(cp, v);
              gst(tk.Cm + col + row * tk.ldc, v);
            }
          } else {
            gst(cp, v);
            if (tk.mirror) gst(tk.Cm + col + row * tk.ldc, tk.mirror == 2 ? 0.0 : v);
          }
        }
      }
    }
}

// Layout of the 64-wide product phases: 0 the 64-tile kernel with the side
// phase in the same launch, 1 / 2 / 3 the product kernel with direct loads
// (layouts 6 / 7 / 8) and the side phase in the same launch, 4 layout 6 or 7
// by the size of the launch, 5 layout 9; INLA_SMALL_VARIANT=0..5 in the
// environment overrides the engine's choice.
static int g_small_variant = kDefaultSmallVariant;
void set_small_variant(int v) {
  g_small_variant = (v >= 0 && v < kSmallVariants) ? v : kDefaultSmallVariant;
}
int small_variant() {
  const char *e = getenv("INLA_SMALL_VARIANT");
  if (e && e[0] >= '0' && e[0] < '0' + kSmallVariants) return e[0] - '0';
  return g_small_variant;
}

// Layout of the 128-wide product kernel: the engine's choice (the autotuner's, else
// the default); INLA_BIG_VARIANT=0..5 in the environment overrides it.
static int g_big_variant = kDefaultBigVariant;
void set_big_variant(int v) {
  g_big_variant = (v >= 0 && v < kBigVariants) ? v : kDefaultBigVariant;
}
int big_variant() {
  const char *e = getenv("INLA_BIG_VARIANT");
  if (e && e[0] >= '0' && e[0] < '0' + kBigVariants) return e[0] - '0';
  return g_big_variant;
}

// C = beta C + sum of the ks partial products of a split-k launch, one
// workgroup per 128-wide tile, with the task's mirroring rules.
__global__ __launch_bounds__(256) void splitk_reduce_kernel(const ItemDev *__restrict__ items,
                                                            int n_items, int phase, int t, int ks) {
  int q = xcd_contiguous(blockIdx.x, gridDim.x);
  const int ii = find_item(items, n_items, q,
                           [&](const ItemDev &x) { return phase_tasks(x, phase, t, 0, true); });
  if (ii >= n_items) return;
  const ItemDev it = items[ii];
  Task tk;
  decode_big<kBig>(it, phase, t, q, tk);
  if (tk.kind != TK_PRODUCT) return;
  const long long bb = (long long)it.b * it.b;
  const double *Pp = it.P + (long long)tk.ti * kBig + (long long)tk.tj * kBig * it.b;
  for (int e = threadIdx.x; e < kBig * kBig; e += 256) {
    const int row = e & (kBig - 1), col = e / kBig;
    if (row >= tk.m || col >= tk.n) continue;
    double v = 0.0;
    for (int h = 0; h < ks; ++h) v += gld(Pp + h * bb + row + (long long)col * it.b);
    double *cp = tk.C + row + (long long)col * tk.ldc;
    if (tk.beta != 0.0) v += tk.beta * gld(cp);
    if (tk.mirror && tk.diagtile) {
      if (row >= col) {
        gst(cp, v);
        gst(tk.Cm + col + (long long)row * tk.ldc, v);
      }
    } else {
      gst(cp, v);
      if (tk.mirror) gst(tk.Cm + col + (long long)row * tk.ldc, v);
    }
  }
}

// Direct-load layouts of the product phases' operands: rows of S, W2 and D
// (layout P) in the factorization; Sigma_{t+1} D rows against inv(L) columns
// in V and the S row of Sigma (P, Q); inv(L) and workspace columns (Q, Q)
// for the diagonal of Sigma.
inline int big_layouts(int phase) {
  switch (phase) {
    case PH_SI_VU_X: case PH_SI_VU_B: case PH_SI_SR_X: return 2;
    case PH_SI_SD_X: case PH_SI_G_B: return 3;
    default: return 0;
  }
}
template <int V>
void launch_big_dma(int phase, int phase2, int nside, long long grid, hipStream_t s,
                    const ItemDev *items_dev, int n_items, int t, int ks) {
  switch (big_layouts(phase)) {
    case 2:
      hipLaunchKernelGGL((tile_product_kernel<V, 2>), dim3((unsigned)grid), dim3(big_threads<V>()), 0, s,
                         items_dev, n_items, phase, phase2, nside, t, ks);
      break;
    case 3:
      hipLaunchKernelGGL((tile_product_kernel<V, 3>), dim3((unsigned)grid), dim3(big_threads<V>()), 0, s,
                         items_dev, n_items, phase, phase2, nside, t, ks);
      break;
    default:
      hipLaunchKernelGGL((tile_product_kernel<V, 0>), dim3((unsigned)grid), dim3(big_threads<V>()), 0, s,
                         items_dev, n_items, phase, phase2, nside, t, ks);
  }
}

hipError_t launch_tile_phase(const ItemDev *items_dev, int n_items, int total, int phase,
                             int phase2, int t, int p, bool big, hipStream_t s, int ks, int nside) {
  if (total <= 0) return hipSuccess;
  // the product kernel: 128-wide tiles, or 64-wide ones in a direct-load form;
  // a side phase rides along only without split-k (total counts its tasks too)
  const bool prod = phase_is_product_x(phase) && (big || small_variant() > 0) &&
                    (phase2 < 0 || ks == 1);
  if (prod) {
    const int nsp = (phase2 >= 0) ? ((nside + 7) & ~7) : 0;
    const int ph2 = (phase2 >= 0) ? phase2 : -1;
    const int ns = (phase2 >= 0) ? nside : 0;
    const long long grid = (long long)(total - ns) * ks + nsp;
    if (!big) {
      int sv = small_variant();
      if (sv == 4) {
        // layout 6 (two workgroups per CU) unless the launch would need a
        // second round of them; then layout 7 (four per CU) fits it in one
        static int cus = 0;
        if (cus == 0) {
          int dev = 0;
          if (hipGetDevice(&dev) != hipSuccess ||
              hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
              cus <= 0)
            cus = 256;
        }
        sv = (grid > 2LL * cus) ? 2 : 1;
      }
      if (sv == 5) launch_big_dma<9>(phase, ph2, ns, grid, s, items_dev, n_items, t, 1);
      else if (sv == 3) launch_big_dma<8>(phase, ph2, ns, grid, s, items_dev, n_items, t, 1);
      else if (sv == 2) launch_big_dma<7>(phase, ph2, ns, grid, s, items_dev, n_items, t, 1);
      else launch_big_dma<6>(phase, ph2, ns, grid, s, items_dev, n_items, t, 1);
      return hipGetLastError();
    }
    switch (big_variant()) {
      case 5: launch_big_dma<5>(phase, ph2, ns, grid, s, items_dev, n_items, t, ks); break;
      case 4: launch_big_dma<4>(phase, ph2, ns, grid, s, items_dev, n_items, t, ks); break;
      case 3: launch_big_dma<3>(phase, ph2, ns, grid, s, items_dev, n_items, t, ks); break;
      case 2:
        hipLaunchKernelGGL(tile_product_kernel<2>, dim3((unsigned)grid), dim3(big_threads<2>()), 0, s,
                           items_dev, n_items, phase, ph2, ns, t, ks);
        break;
      case 1:
        hipLaunchKernelGGL(tile_product_kernel<1>, dim3((unsigned)grid), dim3(big_threads<1>()), 0, s,
                           items_dev, n_items, phase, ph2, ns, t, ks);
        break;
      default:
        hipLaunchKernelGGL(tile_product_kernel<0>, dim3((unsigned)grid), dim3(big_threads<0>()), 0, s,
                           items_dev, n_items, phase, ph2, ns, t, ks);
    }
    if (ks > 1) {
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(splitk_reduce_kernel, dim3(total), dim3(256), 0, s, items_dev, n_items,
                         phase, t, ks);
    }
  } else if (phase_is_fat(phase) || (phase2 >= 0 && phase_is_fat(phase2))) {
    // the Cholesky-capable kernel decodes its own phases only
    if (!phase_is_fat(phase) || (phase2 >= 0 && !phase_is_fat(phase2))) return hipErrorInvalidValue;
    hipLaunchKernelGGL(tile_phase_kernel<true>, dim3(total), dim3(kThreads), 0, s, items_dev, n_items,
                       phase, phase2, t, p);
  } else {
    hipLaunchKernelGGL(tile_phase_kernel<false>, dim3(total), dim3(kThreads), 0, s, items_dev,
                       n_items, phase, phase2, t, p);
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

// Stores one item descriptor, passed by value as a kernel argument, into
// device memory (no host staging buffer: nothing is read from host memory
// when the copy runs).
__global__ void put_item_kernel(ItemDev it, ItemDev *dst) {
  if (threadIdx.x == 0) *dst = it;
}

hipError_t launch_put_item(const ItemDev &it, ItemDev *dst, hipStream_t s) {
  hipLaunchKernelGGL(put_item_kernel, dim3(1), dim3(64), 0, s, it, dst);
  return hipGetLastError();
}

// log|Q| = 2 sum of the per-tile partial sums of log L_jj, in a fixed tree order.
// Item i writes logdet_out[i * stride] and info_out[i * stride].
__global__ void logdet_finish_kernel(const ItemDev *items, double *logdet_out, int *info_out,
                                     int stride) {
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
    if (info_out) info_out[blockIdx.x * stride] = (inf == kInfoNone) ? 0 : inf;
    if (logdet_out) logdet_out[blockIdx.x * stride] = (inf == kInfoNone) ? 2.0 * red[0] : NAN;
  }
}

hipError_t launch_logdet_finish(const ItemDev *items_dev, int n_items, double *logdet_out,
                                int *info_out, hipStream_t s, int stride) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(logdet_finish_kernel, dim3(n_items), dim3(256), 0, s, items_dev, logdet_out,
                     info_out, stride);
  return hipGetLastError();
}

}  // namespace inla
