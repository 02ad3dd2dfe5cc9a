// Internal declarations shared by the device kernels and the host engine.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/inla_bta.h"

namespace inla {

constexpr int kTile = 64;        // tile edge of the block kernels (rows = cols)
constexpr int kMaxArrow = 64;    // arrow (fixed-effect) width handled by one tile
constexpr int kThreads = 256;    // threads per workgroup of the tile kernels
constexpr int kInfoNone = 0x7fffffff;

// Device view of one model (read-only after create).
struct ModelDev {
  int N, nt, a, b;               // grid side, time steps, arrow width, block size N*N
  long long m;                   // observations
  long long n;                   // latent dimension b*nt + a
  double h, beta_prec;
  double prior_mean[4], prior_prec[4];
  // union pattern of Q_s and of every A_t^T A_t, column-compressed over b x b
  int nnz;
  int sbw;                       // half-bandwidth of Q_s: entries with |r - c| > sbw are zero
  const int *colptr;             // b + 1
  const int *rowidx;             // nnz
  const int *colidx;             // nnz: column of each pattern entry
  const double *pdelta;          // nnz: identity entry (1 on the diagonal)
  const double *pg1;             // nnz: grid Laplacian G
  const double *pg2;             // nnz: G^2
  const double *AtA;             // nt * nnz: (A_t^T A_t) on the pattern
  const double *ZtA;             // nt * a * b: (Z^T A_t), column-major a x b per t
  const double *ZtZ;             // a * a
  const double *Aty;             // n: A^T y
  const long long *A_rowptr;     // m + 1
  const int *A_col;              // nnz(A)
  const double *A_val;
  const double *y;               // m
  // A by columns (row indices ascending within a column, duplicates summed)
  // and its fixed-effect columns dense: for likelihoods whose A^T diag(d) A
  // is assembled anew for every d
  const long long *Ac_ptr;       // n + 1
  const int *Ac_row;             // nnz of the CSC form
  const double *Ac_val;
  const double *Zd;              // m x a, row-major
};

// Device descriptor of one BTA matrix in flight through factor / selinv.
struct ItemDev {
  int b, nt, a, nP;              // block size, time blocks, arrow width, ceil(b / kTile)
  double *D, *S, *R, *T;         // BTA storage (Q in, factor out)
  double *W1, *W2, *W3;          // workspace: b*b (running sums of inv(L_tt) rows in the
                                 // factorization, Sigma_S in the selected inversion),
                                 //   b*b (panels of L_tt, then S[t] Linv^T), a*b
  double *Mp;                    // 2 x 64 x 64: M_p = inv(A_pp) of the current diagonal tile,
                                 // by parity (the batched Cholesky step reads it)
  double *P;                     // kSplitK * b * b split-k partial products (or null: no split)
  // Selected inversion with every step's V_t = L_{t+1,t} inv(L_tt) ((nt-1) b*b),
  // U_t = L_{A,t} inv(L_tt) (nt a*b) and G_t = inv(L_tt)^T inv(L_tt) (nt b*b,
  // lower tiles) formed up front, in one launch each (null: V_t and U_t are
  // formed step by step in W2 and W3, G_t inside the step's Sigma_D[t] launch).
  double *V, *U, *G;
  // Selected inversion: Sigma blocks.  When sd_stride != 0 the blocks of step t
  // live at SD + t*sd_stride etc. (caller storage); otherwise Sigma_D and
  // Sigma_R ping-pong between two buffers by the parity of t and Sigma_S uses
  // one buffer.
  double *SD, *SS, *SR, *ST;
  long long sd_stride, ss_stride, sr_stride;
  double *ldpart;                // nt*nP + 1 partial sums of log L_jj
  int *info;                     // first failing pivot (1-based row); kInfoNone = none
  // outputs of the selected inversion
  double *diag;                  // n marginal variances (or null)
  double *trpart;                // (nt + 1) * kTraceBlocks * 4 partial traces (or null)
  const ModelDev *model;         // model whose derivative blocks the traces use (or null)
  const double *theta;           // 4 hyperparameters of this item (device)
  int which;                     // 0: Q_prior, 1: Q_c
  // Two-sided elimination.  An item is a chain of nt time blocks of a matrix
  // with ntf blocks: step t of the chain is time block tmap(t) = t (trev = 0)
  // or ntf - 1 - t (trev = 1: the chain runs from the last block backwards,
  // reading each coupling block as its transpose).  The chain runs steps
  // t < nrun (nrun = nt, or nt - 1 for a backward chain whose last block is
  // the middle block, factored by the forward chain).  own_arrow: the item
  // factors / inverts the arrow block itself (a whole matrix); a half never does.
  int ntf, trev, nrun, own_arrow;
  // Half-bandwidth of the coupling blocks S[t] (entries with |r - c| > sbw
  // are zero; b when they are dense).  Then X = S[t] inv(L_tt)^T = L_{t+1,t}
  // has zeros left of column r - sbw in row r (upper trapezoidal), and the
  // products that read S[t] or X skip the k ranges of those zeros.
  int sbw;
};

// Time block of chain step t, and the storage of the chain's blocks.  The
// coupling of backward-chain steps t and t+1 (times tau and tau - 1) is stored
// in the forward slot of block (tau, tau - 1), which holds its transpose.
__host__ __device__ inline int tmap(const ItemDev &it, int t) { return it.trev ? it.ntf - 1 - t : t; }
__host__ __device__ inline double *dblk(const ItemDev &it, int t) {
  return it.D + (long long)tmap(it, t) * it.b * it.b;
}
__host__ __device__ inline double *sblk(const ItemDev &it, int t) {
  return it.S + (long long)(tmap(it, t) - it.trev) * it.b * it.b;
}
__host__ __device__ inline double *rblk(const ItemDev &it, int t) {
  return it.R + (long long)tmap(it, t) * it.a * it.b;
}

__host__ __device__ inline double *sig_D(const ItemDev &it, int t) {
  return it.sd_stride ? it.SD + (long long)t * it.sd_stride : it.SD + (long long)(t & 1) * it.b * it.b;
}
__host__ __device__ inline double *sig_S(const ItemDev &it, int t) {
  return it.ss_stride ? it.SS + (long long)t * it.ss_stride : it.SS;
}
__host__ __device__ inline double *sig_R(const ItemDev &it, int t) {
  return it.sr_stride ? it.SR + (long long)t * it.sr_stride : it.SR + (long long)(t & 1) * it.a * it.b;
}

// Phases of the tile kernels.  Phases ending in _X are the b x b products; they
// run either on 64 x 64 tiles or on 128 x 128 "big" tiles (big = true).
enum Phase : int {
  PH_DIAG0 = 0,      // Cholesky + inverse of tile (0,0) of D[t]
  PH_STEP = 1,       // step p = 0..nP-1 of the tile Cholesky and of inv(L_tt) (with lookahead):
                     //   panel p: L[i,p] = A[i,p] X_pp^T into W2 (i > p),
                     //   column p+1 below the diagonal: A[i,p+1] -= L[i,p-1] L[p+1,p-1]^T
                     //     + (A[i,p] M_p) A[p+1,p]^T with M_p = inv(A_pp) (i > p+1),
                     //   the rest of panel p-1's update: A[i,j] -= L[i,p-1] L[j,p-1]^T (j > p+1),
                     //   row p of X = inv(L_tt): X[p,j] = -X_pp sum_{j<=m<p} L[p,m] X[m,j] (j < p)
  PH_DIAGC = 2,      // beside STEP(p): tile (p+1,p+1) updated as its column, then its
                     //   Cholesky + inverse and M_{p+1}
  PH_STEPF = 3,      // DIAGC(p) and STEP(p) as one launch of the Cholesky-capable kernel
                     //   (few tasks per step: the launch latency dominates); the column-p
                     //   term of column p+1 is L[i,p] L[p+1,p]^T formed in the task from
                     //   X_pp, so no M_p is needed
  PH_OFFDIAG_X = 4,  // X = S[t] Linv^T
  PH_OFFDIAG = 5,    // R' = R[t] Linv^T
  PH_SCHUR_X = 6,    // D[t+1] -= X X^T
  PH_SCHUR = 7,      // R[t+1] -= R' X^T, T -= R' R'^T; copy X, R' back
  PH_ARROW = 8,      // Cholesky + inverse of T
  PH_SI_INIT = 9,    // Sigma_T = Linv_AA^T Linv_AA
  PH_SI_VU_X = 10,   // V = L_{t+1,t} Linv_tt
  PH_SI_VU = 11,     // U = L_{A,t} Linv_tt
  PH_SI_SR_X = 12,   // Sigma_S[t]
  PH_SI_SR = 13,     // Sigma_R[t]
  PH_SI_SD_X = 14,   // Sigma_D[t] (lower tiles, mirrored)
  PH_SI_VU_B = 15,   // V_t for every t < nt-1 into V (one launch; V_t needs only the factor)
  PH_SI_U_B = 16,    // U_t for every t into U
  PH_SI_G_B = 17,    // G_t = inv(L_tt)^T inv(L_tt) for every t into G (lower tiles)
  PH_COUNT = 18
};

constexpr int kTraceBlocks = 16;   // workgroups per item in a trace reduction step
constexpr int kBig = 128;        // edge of a big tile
__host__ __device__ inline int nbig(int n) { return (n + kBig - 1) / kBig; }
__host__ __device__ inline bool phase_is_product_x(int phase) {
  return phase == PH_OFFDIAG_X || phase == PH_SCHUR_X || phase == PH_SI_VU_X ||
         phase == PH_SI_SR_X || phase == PH_SI_SD_X || phase == PH_SI_VU_B || phase == PH_SI_G_B;
}

__host__ __device__ inline int ntile(int n) { return (n + kTile - 1) / kTile; }

// The tasks of a Cholesky step launch (PH_STEP, PH_STEPF) of one item in two
// classes: long ones (the diagonal tile, the chained tasks of column p+1 and
// of the diagonal tile of column p+2, row p of inv(L_tt)) and short ones
// (single products: panels, the rest of panel p-1's update, running sums).
// step_task_local maps an index within a class to the item's task index in
// the decoder's order (diagonal tile, panels, chained tasks, deferred
// updates, rows, running sums).
struct StepSplit {
  int ndiag, npan, ncol, ndef, nrow, nsum;
  __host__ __device__ int nlong() const { return ndiag + ncol + (ndef > 0 ? 1 : 0) + nrow; }
  __host__ __device__ int nshort() const { return npan + ndef - (ndef > 0 ? 1 : 0) + nsum; }
};
__host__ __device__ inline StepSplit step_split(int nP, int phase, int t, int p, int nrun) {
  StepSplit z{0, 0, 0, 0, 0, 0};
  if (t >= nrun || p >= nP) return z;
  z.npan = nP - 1 - p;
  z.ncol = (nP - 2 - p > 0) ? nP - 2 - p : 0;
  // the batched step is left-looking: no deferred trailing tiles
  z.ndef = (phase == PH_STEP) ? 0 : (p >= 1) ? z.ncol * (z.ncol + 1) / 2 : (z.ncol > 0 ? 1 : 0);
  z.nrow = p;
  z.nsum = (phase == PH_STEPF) ? (nP - 1 - p) * p : 0;
  z.ndiag = (phase == PH_STEPF && p < nP - 1) ? 1 : 0;
  return z;
}
__host__ __device__ inline int step_task_local(const StepSplit &z, bool is_long, int c) {
  const int d1 = z.ndef > 0 ? 1 : 0;
  if (is_long) {
    if (c < z.ndiag) return 0;
    c -= z.ndiag;
    if (c < z.ncol) return z.ndiag + z.npan + c;
    c -= z.ncol;
    if (c < d1) return z.ndiag + z.npan + z.ncol;   // deferred task 0: the chained diagonal tile
    c -= d1;
    return z.ndiag + z.npan + z.ncol + z.ndef + c;
  }
  if (c < z.npan) return z.ndiag + c;
  c -= z.npan;
  if (c < z.ndef - d1) return z.ndiag + z.npan + z.ncol + d1 + c;
  c -= z.ndef - d1;
  return z.ndiag + z.npan + z.ncol + z.ndef + z.nrow + c;
}

// Number of workgroup tasks of one item in (phase, t, p); big selects 128-tiles
// for the _X phases.
__host__ __device__ inline int phase_tasks(const ItemDev &it, int phase, int t, int p,
                                           bool big = false) {
  const int nP = it.nP;
  const int nQ = big ? nbig(it.b) : nP;
  const bool arrow = it.a > 0;
  if (phase == PH_ARROW || phase == PH_SI_INIT) return (arrow && it.own_arrow) ? 1 : 0;
  // the every-step phases count from the launch's t = 0 over the chain's steps
  if (phase == PH_SI_VU_B) return (it.nrun < it.nt ? it.nrun : it.nt - 1) * nQ * nQ;
  if (phase == PH_SI_U_B) return arrow ? it.nrun * nP : 0;
  if (phase == PH_SI_G_B) return it.nrun * (nQ * (nQ + 1) / 2);
  if (t >= it.nrun) return 0;
  const bool last = (t == it.nt - 1);
  switch (phase) {
    case PH_DIAG0: return 1;
    case PH_STEP:     // panels, column p+1 (left-looking: every earlier panel), row p of inv(L_tt)
    case PH_STEPF: {  // panels, column p+1, the deferred trailing tiles (right-looking),
                      // row p of inv(L_tt), the diagonal tile of column p+1 and the running
                      // sums of the later rows of inv(L_tt)
      if (p >= nP) return 0;
      const int ncol = (nP - 2 - p > 0) ? nP - 2 - p : 0;
      const int ndef = (phase == PH_STEP) ? 0 : (p >= 1 ? ncol * (ncol + 1) / 2 : (ncol > 0 ? 1 : 0));
      return (nP - 1 - p) + ncol + ndef + p +
             ((phase == PH_STEPF) ? (nP - 1 - p) * p : 0) +
             ((phase == PH_STEPF && p < nP - 1) ? 1 : 0);
    }
    case PH_DIAGC: return (p < nP - 1) ? 1 : 0;
    case PH_OFFDIAG_X: return last ? 0 : nQ * nQ;
    case PH_OFFDIAG: return arrow ? nP : 0;
    case PH_SCHUR_X: return last ? 0 : nQ * (nQ + 1) / 2;
    case PH_SCHUR:
      return (last ? 0 : nP * nP) + (arrow ? ((last ? 0 : nP) + 1 + nP) : 0);
    case PH_SI_VU_X: return last ? 0 : nQ * nQ;
    case PH_SI_VU: return arrow ? nP : 0;
    case PH_SI_SR_X: return last ? 0 : nQ * nQ;
    case PH_SI_SR: return arrow ? nP : 0;
    case PH_SI_SD_X: return nQ * (nQ + 1) / 2;
    default: return 0;
  }
}

// Phases whose workgroups may run the in-tile Cholesky (large-LDS variant).
__host__ __device__ inline bool phase_is_fat(int phase) {
  return phase == PH_DIAG0 || phase == PH_DIAGC || phase == PH_STEPF || phase == PH_ARROW;
}

// Sets the calling thread's inla_last_error() text and returns st.
inla_status set_last_error(inla_status st, const char *msg);
// ---- launch wrappers (bta_kernels.hip) ----
// total counts the tasks of both phases; with the product kernel (big, or a
// direct-load 64-wide form) and phase2 >= 0, nside of them are phase2's and
// ks must be 1.
hipError_t launch_tile_phase(const ItemDev *items_dev, int n_items, int total, int phase,
                             int phase2, int t, int p, bool big, hipStream_t s, int ks = 1,
                             int nside = 0);
constexpr int kSplitK = 2;        // k-split of 128-tile launches with too few tiles
hipError_t launch_fill(double *ptr, long long n, double v, hipStream_t s);
hipError_t launch_fill_int(int *ptr, long long n, int v, hipStream_t s);
// Writes *dst = it on the stream (the descriptor travels as a kernel argument).
hipError_t launch_put_item(const ItemDev &it, ItemDev *dst, hipStream_t s);
hipError_t launch_logdet_finish(const ItemDev *items_dev, int n_items, double *logdet_out,
                                int *info_out, hipStream_t s, int stride = 1);
// Layout of the 128-wide tile kernel (0: 8 waves of 64 x 32, k-chunk 16, two
// register sets; 1: 4 waves of 64 x 64; 2: as 0 with k-chunk 32, one set;
// 3, 4: 8 waves of 64 x 32 staged by direct loads into LDS, k-chunk 32 / 16,
// the latter two workgroups per compute unit; 5: 4 waves of 64 x 64, direct
// loads, k-chunk 16, two workgroups per compute unit).
constexpr int kBigVariants = 6;
constexpr int kDefaultBigVariant = 4;
// Form of the 64-wide product phases (0: 64-tile kernel, the side phase in the
// same launch; 1, 2, 3: product kernel with direct loads, k-chunk 32 / 16 /
// 16 with four LDS stages; 4: 1, or 2 when a launch has more workgroups than
// two per compute unit; 5: as 2 on eight waves of 32 x 16, the same sums in
// the same order).
constexpr int kSmallVariants = 6;
constexpr int kDefaultSmallVariant = 5;
void set_small_variant(int v);
int small_variant();
void set_big_variant(int v);
int big_variant();
// ---- model kernels (model_kernels.hip) ----
// Assemble Q_prior (which = 0) or Q_c (which = 1) of one model into BTA storage;
// with rhs != null also b = tau_y A^T y.
hipError_t launch_assemble(const ModelDev *model_dev, int b, int nt, int a, const double *theta,
                           int which, double *D, double *S, double *R, double *T, double *rhs,
                           hipStream_t s);
// One stage of the forward / backward substitution sweeps for a batch of
// factors.  xs[i] (n_i doubles, device) holds the right-hand side on entry and
// the solution on exit; tmps[i] is max(b_i, a_i) doubles of scratch.
enum SolveStage : int { SV_F1 = 0, SV_F2 = 1, SV_FA1 = 2, SV_FA2 = 3, SV_BA = 4, SV_B1 = 5, SV_B2 = 6 };
hipError_t launch_solve_stage(const ItemDev *items_dev, int n_items, int max_b, int max_a, int t,
                              int stage, double *const *xs_dev, double *const *tmps_dev,
                              hipStream_t s);
// Traces of Sigma with the derivative blocks and the marginal variances of
// time block t (t = -1: the arrow block).
hipError_t launch_trace_step(const ItemDev *items_dev, int n_items, int t, hipStream_t s);
// Posterior-mode terms: per item partial sums of mu^T Q_st mu, mu^T dQ2 mu,
// mu^T dQ3 mu and |y - A mu|^2 (beta part included in the first).
constexpr int kTermBlocks = 256;
struct TermItem {
  const ModelDev *model;
  const double *theta;   // 4
  const double *mu;      // n
  double *part;          // kTermBlocks * 4
};
hipError_t launch_terms(const TermItem *items_dev, int n_items, hipStream_t s);
// Final combination: f and gradient of each theta item.
struct CombineItem {
  const ModelDev *model;
  const double *theta;
  const double *term_part;   // kTermBlocks * 4
  const double *mu;          // n (posterior mode)
  const double *logdet;      // [0] = log|Q_p|, [1] = log|Q_c|
  const double *trp;         // (nt + 1) * kTraceBlocks * 4 partial traces of Q_p (or null)
  const double *trc;         // (nt + 1) * kTraceBlocks * 4 partial traces of Q_c (or null)
  const int *info;           // [0] Q_p, [1] Q_c
  double *f;                 // 1
  double *grad;              // 4 (or null)
  int *status;               // 1 (or null)
  int pad_;
};
hipError_t launch_combine(const CombineItem *items_dev, int n_items, hipStream_t s);
// A matrix eliminated from both ends (a forward chain over time blocks 0..m,
// a backward chain from block nt-1 down to m+1): the backward chain's arrow
// updates collect in TB, and the middle block's selected-inverse blocks are
// handed from the forward chain's buffers to the backward chain's.
struct TwistPair {
  double *T, *TB;          // arrow block (a x a) and the backward chain's accumulator
  const double *SDf;       // Sigma of the middle block in the forward chain's buffer (b x b)
  double *SDb;             // ... and where the backward chain reads it
  const double *SRf;       // Sigma_{A,m} (a x b), likewise
  double *SRb;
  int a, b, m;             // arrow width, block size, middle block
  int pad_;
};
// Accessors of a model (engine.cpp): its device descriptor, the host copy of
// that descriptor (device pointers inside), and whether every y_i is a count
// (with sum_i log y_i!).
const ModelDev *model_device(const inla_model *m);
const ModelDev &model_host_desc(const inla_model *m);
bool model_counts(const inla_model *m, double *log_y_fact);

// Poisson likelihood (the inner Newton loop), kNgBlocks partial sums each:
//   ng_obs:   eta = A x, e = exp(eta) (e_out), w = y + e (eta - 1) (w_out; both
//             may be null), part[k] = partial sums of y_i eta_i - e_i;
//   ng_atv:   out = A^T v (n = nst + a: the space-time columns, then the a
//             fixed-effect columns, each reduced by a workgroup);
//   ng_add_obs: D[t] += (A^T diag(e) A) on the pattern, R[t] += its fixed-effect
//             rows, T += Z^T diag(e) Z (BTA storage of the model's shape);
//   ng_obs_var: c_i = 1/2 e_i (A Sigma A^T)_ii from Sigma's D, R, T blocks;
//   ng_quad:  part[4k..] = u^T Q_st v, u^T dQ_st/dtheta_2 v, u^T dQ_st/dtheta_3 v,
//             u_beta^T v_beta;
//   ng_step:  cand = x + step (xn - x), part[2k..] = max |cand - x|, max |x|.
constexpr int kNgBlocks = 256;
hipError_t launch_ng_obs(const ModelDev *M, long long m, const double *x, double *e_out, double *w_out,
                         double *part, hipStream_t s);
hipError_t launch_ng_atv(const ModelDev *M, long long nst, int a, const double *v, double *out,
                         hipStream_t s);
hipError_t launch_ng_add_obs(const ModelDev *M, int b, int nt, int a, int nnz, const double *e, double *D,
                             double *R, double *T, hipStream_t s);
hipError_t launch_ng_obs_var(const ModelDev *M, long long m, const double *SD, const double *SR,
                             const double *ST, const double *e, double *c_out, hipStream_t s);
hipError_t launch_ng_quad(const ModelDev *M, const double *theta, const double *u, const double *v,
                          double *part, hipStream_t s);
hipError_t launch_ng_step(const double *x, const double *xn, double step, double *cand, long long n,
                          double *part, hipStream_t s);

// Mixture of K Gaussians N(mu^k, v^k) with weights w (device, K doubles; mu, var:
// K x n point-major).  With d = mu^k - shift: acc_m (+)= sum_k w_k d,
// acc_s (+)= sum_k w_k (v^k + d^2) (init = 1 starts from zero).  The finish
// writes mean = shift + acc_m and var = acc_s - acc_m^2 (weights summing to 1).
hipError_t launch_mixture_accumulate(const double *mu, const double *var, const double *w, int K,
                                     long long n, const double *shift, double *acc_m, double *acc_s,
                                     int init, hipStream_t s);
hipError_t launch_mixture_finish(const double *shift, const double *acc_m, const double *acc_s,
                                 long long n, double *mean_out, double *var_out, hipStream_t s);
// mode 0: TB = 0; mode 1: T += TB.
hipError_t launch_twist_arrow(const TwistPair *pairs_dev, int n_pairs, int max_a, int mode,
                              hipStream_t s);
// For the pairs whose middle block is m == t: SDb = SDf, SRb = SRf.
hipError_t launch_twist_middle(const TwistPair *pairs_dev, int n_pairs, int max_b, int max_a, int t,
                               hipStream_t s);

}  // namespace inla
