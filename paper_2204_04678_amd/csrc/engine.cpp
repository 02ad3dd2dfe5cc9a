// Host engine and C ABI of the BTA INLA library (see include/inla_bta.h).
//
// The engine turns each ABI call into a fixed sequence of batched kernel
// launches on the caller's stream:
//   factor   (per time step t, all items in lockstep)
//       DIAG0, then for each 64-wide tile p one STEP(p) launch (panel p of L,
//       the lookahead update of column p+1, the rest of panel p-1's update,
//       row p of inv(L_tt) written in place into D[t]) with the Cholesky +
//       inverse of tile p+1 fused or beside it; then OFFDIAG (X = S[t]
//       inv(L_tt)^T, R' = R[t] inv(L_tt)^T) and SCHUR (D[t+1] -= X X^T,
//       R[t+1] -= R' X^T, T -= R' R'^T); finally ARROW.
//   selected inversion (t = nt-1 .. 0), the block form of the Takahashi
//   recursion (paper, Sec. "Partial Inversion"), derived from Sigma L = L^{-T}
//   read block column by block column:
//       V = L_{t+1,t} inv(L_tt), U = L_{A,t} inv(L_tt)
//       Sigma_{t+1,t} = -(Sigma_{t+1,t+1} V + Sigma_{A,t+1}^T U)
//       Sigma_{A,t}   = -(Sigma_{A,t+1} V + Sigma_{AA} U)
//       Sigma_{t,t}   = inv(L_tt)^T inv(L_tt) - Sigma_{t+1,t}^T V - Sigma_{A,t}^T U
//   and per step the trace reductions against the derivative blocks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/inla_bta.h"
#include "graph_key.h"
#include "inla_internal.h"

using namespace inla;

namespace {

thread_local std::string g_last_error;

inla_status fail(inla_status st, const std::string &msg) {
  g_last_error = msg;
  return st;
}

}  // namespace

namespace inla {
inla_status set_last_error(inla_status st, const char *msg) {
  g_last_error = msg ? msg : "";
  return st;
}
}  // namespace inla

namespace {

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail(INLA_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));          \
  } while (0)

// ---------------------------------------------------------------------------
// device workspace arena: one allocation, carved per call, grown on demand
// ---------------------------------------------------------------------------
struct Arena {
  char *base = nullptr;
  size_t cap = 0;
  int device = -1;
  hipEvent_t last = nullptr;  // completion of the last call that used the arena
  hipStream_t last_stream = nullptr;
  unsigned long long gen = 0; // bumped whenever a call lays out the arena afresh
};
std::mutex g_mutex;
Arena g_arena;

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Collects sub-allocation requests, then binds them into the arena.
struct Layout {
  struct Req { void **slot; size_t bytes; };
  std::vector<Req> reqs;
  size_t total = 0;
  template <class T>
  void add(T **slot, size_t count) {
    reqs.push_back({reinterpret_cast<void **>(slot), count * sizeof(T)});
    total += align_up(std::max<size_t>(count * sizeof(T), 1));
  }
};

inla_status arena_bind(Layout &L, hipStream_t s) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (g_arena.base && g_arena.device != dev) {
    return fail(INLA_ERR_STATE, "library workspace is bound to another device");
  }
  // order this call after the previous user of the arena
  if (g_arena.last && g_arena.last_stream != s) HIP_TRY(hipStreamWaitEvent(s, g_arena.last, 0));
  if (L.total > g_arena.cap) {
    if (g_arena.base) {
      HIP_TRY(hipDeviceSynchronize());
      HIP_TRY(hipFree(g_arena.base));
      g_arena.base = nullptr;
      g_arena.cap = 0;
    }
    size_t want = align_up(L.total);
    void *p = nullptr;
    if (hipMalloc(&p, want) != hipSuccess) {
      (void)hipGetLastError();
      return fail(INLA_ERR_NOMEM, "device workspace allocation of " + std::to_string(want) +
                                      " bytes failed");
    }
    g_arena.base = static_cast<char *>(p);
    g_arena.cap = want;
    g_arena.device = dev;
  }
  size_t off = 0;
  for (auto &r : L.reqs) {
    *r.slot = g_arena.base + off;
    off += align_up(std::max<size_t>(r.bytes, 1));
  }
  ++g_arena.gen;
  return INLA_OK;
}

inla_status arena_done(hipStream_t s) {
  if (!g_arena.last) HIP_TRY(hipEventCreateWithFlags(&g_arena.last, hipEventDisableTiming));
  HIP_TRY(hipEventRecord(g_arena.last, s));
  g_arena.last_stream = s;
  return INLA_OK;
}

template <class T>
inla_status upload(T *dst, const std::vector<T> &src, hipStream_t s) {
  if (src.empty()) return INLA_OK;
  HIP_TRY(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s));
  return INLA_OK;
}

// ---------------------------------------------------------------------------
// phase sequences
// ---------------------------------------------------------------------------
bool use_big_tiles(const std::vector<ItemDev> &items);

struct Batch {
  std::vector<ItemDev> host;
  ItemDev *dev = nullptr;
  int max_nt = 0, max_b = 0, max_a = 0;
  bool big = false;
  bool split = false;   // every item has split-k scratch
  bool vb = false;      // selected inversion with V_t, U_t of every step formed up front
  void finalize() {
    big = use_big_tiles(host);
    split = !host.empty();
    for (auto &it : host) split = split && it.P;
    for (auto &it : host) {
      max_nt = std::max(max_nt, it.nt);
      max_b = std::max(max_b, it.b);
      max_a = std::max(max_a, it.a);
    }
  }
};

// The products that read the coupling blocks skip the zeros outside their band
// (ItemDev::sbw); INLA_BAND=0 in the environment treats the blocks as dense.
bool band_aware() {
  const char *e = getenv("INLA_BAND");
  return !(e && e[0] == '0');
}

// Multiply-adds of the band-aware b x b products with coupling half-bandwidth
// w (X = S inv(L)^T with S banded and inv(L) lower; the lower half of X X^T;
// V = X inv(L); the arrow rows times X^T), entry by entry:
//   X(r, c):    k from max(0, r - w) to min(c, r + w)
//   XX^T(r, c): k from max(0, r - w) to b - 1 (r >= c)
//   V(r, c):    k from max(c, r - w) to b - 1
//   W X^T(., c): k from max(0, c - w) to b - 1 (per arrow row)
struct BandMacs {
  double x = 0, syrk = 0, v = 0, arrow = 0;
};
BandMacs band_macs(long long b, long long w) {
  BandMacs m;
  for (long long r = 0; r < b; ++r) {
    const long long lo = std::max(0LL, r - w), hi = std::min(b - 1, r + w);
    const long long L = hi - lo + 1;
    m.x += 0.5 * (double)L * (L + 1) + (double)(b - 1 - hi) * L;   // c from lo to b - 1
    m.syrk += (double)(r + 1) * (b - lo);
    m.v += (double)lo * (b - lo) + 0.5 * (double)(b - lo) * (b - lo + 1);
    m.arrow += (double)(b - lo);
  }
  return m;
}

// Algorithmic FP64 flops of one item in one phase (dense-block counts:
// POTRF(b) = b^3/3, TRTRI(b) = b^3/3, TRSM/TRMM(m x b) = m b^2, SYRK(n, k) = n^2 k,
// GEMM(m, n, k) = 2 m n k, LAUUM(b) = b^3/3).
double phase_flops(const ItemDev &it, int phase, int t, int p) {
  if (phase_tasks(it, phase, t, p) == 0) return 0.0;
  const double b = it.b, a = it.a, b3 = b * b * b;
  const bool last = (t == it.nt - 1);
  if (it.sbw < it.b) {
    // the products that meet the band: their band-aware counts
    const BandMacs m = band_macs(it.b, it.sbw);
    switch (phase) {
      case PH_OFFDIAG_X: return last ? 0.0 : 2.0 * m.x;
      case PH_SCHUR_X: return last ? 0.0 : 2.0 * m.syrk;
      case PH_SCHUR: return (last ? 0.0 : 2.0 * a * m.arrow) + a * a * b;
      case PH_SI_VU_X: return last ? 0.0 : 2.0 * m.v;
      case PH_SI_VU_B: return (it.nt - 1) * 2.0 * m.v;
      default: break;
    }
  }
  switch (phase) {
    // POTRF and TRTRI of the block (2 b^3 / 3) spread over its launches: the
    // first diagonal tile, then every tile step equally
    case PH_DIAG0: return 2.0 * b3 / 3.0 / it.nP;
    case PH_STEP:
    case PH_STEPF: return 2.0 * b3 / 3.0 * (it.nP - 1) / ((double)it.nP * it.nP);
    case PH_OFFDIAG_X: return last ? 0.0 : b3;
    case PH_OFFDIAG: return a * b * b;
    case PH_SCHUR_X: return last ? 0.0 : b3;
    case PH_SCHUR: return (last ? 0.0 : 2.0 * a * b * b) + a * a * b;
    case PH_ARROW: return 2.0 * a * a * a / 3.0;
    case PH_SI_INIT: return a * a * a / 3.0;
    case PH_SI_VU_X: return last ? 0.0 : b3;
    case PH_SI_VU: return a * b * b;
    case PH_SI_SR_X: return last ? 0.0 : 2.0 * b3 + 2.0 * a * b * b;
    case PH_SI_SR: return (last ? 0.0 : 2.0 * a * b * b) + 2.0 * a * a * b;
    case PH_SI_SD_X: return (it.G ? 0.0 : b3 / 3.0) + (last ? 0.0 : b3) + a * b * b;
    case PH_SI_VU_B: return (it.nt - 1) * b3;
    case PH_SI_U_B: return it.nt * a * b * b;
    case PH_SI_G_B: return it.nt * b3 / 3.0;
    default: return 0.0;
  }
}

// Tile size of the b x b product phases: the caller's or the autotuner's
// choice (g_tile_pref), else 128-wide tiles when a launch has enough of them
// to fill the chip and 64-wide ones otherwise.  INLA_TILE=64|128 in the
// environment overrides both.
// With split-k scratch (every item has P), 128-tile launches of fewer than
// kSplitTiles tiles split their k range over kSplitK workgroups.  The built-in
// rule picks 128-wide tiles only from kSplitTiles tiles per launch on: below
// that the 64-wide kernel was faster on every workload measured (b = 1024 with
// two matrices, b = 1600 with two), split or not; the autotuner and the tile
// option can still ask for 128 (then split) there.
constexpr long long kSplitTiles = 384;
// Below this many 64-wide tiles per step (over the selected inversion's
// matrices) the V_t, U_t of every step are formed up front, in one launch each.
constexpr long long kVBatchTiles = 4096;
// Below this many 64-tiles (summed nP^2 over the items of a factor launch)
// each Cholesky step is one fused launch (see run_factor).  Measured on
// b = 2025 with 2, 4 and 8 matrices (2048, 4096, 8192 tiles): fused 23%, 11%
// faster and 1% slower per evaluation; b = 1600 with 2 matrices: 13% faster.
constexpr long long kStepFusedTiles = 6144;
// INLA_STEP_FUSED=1 (0) in the environment makes every Cholesky step fused
// (batched); else the autotuner's choice (g_step_pref), else the tile-count rule.
int g_step_pref = -1;
int step_fused_override() {
  const char *e = getenv("INLA_STEP_FUSED");
  return (e && (e[0] == '0' || e[0] == '1')) ? e[0] - '0' : g_step_pref;
}
// INLA_SI_BATCH=0 keeps the selected inversion's V_t, U_t step by step; 1 (or
// unset) forms them up front where the built-in rule wants it.
bool si_batch_allowed() {
  const char *e = getenv("INLA_SI_BATCH");
  return !(e && e[0] == '0');
}
int g_tile_pref = 0;
// The tile size asked for: INLA_TILE in the environment, else the engine's choice.
int tile_request() {
  const char *e = getenv("INLA_TILE");
  return e ? atoi(e) : g_tile_pref;
}
bool use_big_tiles(const std::vector<ItemDev> &items) {
  const int force = tile_request();
  if (force == 64) return false;
  if (force == 128) return true;
  long long big = 0;
  for (const auto &it : items) big += (long long)nbig(it.b) * nbig(it.b);
  return big >= kSplitTiles;
}

#define ST_TRY_INNER(expr)               \
  do {                                   \
    inla_status st_ = (expr);            \
    if (st_ != INLA_OK) return st_;      \
  } while (0)

// Profiling slots: the tile phases, then the other kernel families.
enum ProfSlot : int { PS_SOLVE = PH_COUNT, PS_TRACE, PS_ASSEMBLE, PS_MISC, PS_COUNT };

// Kernel behind a record: 0 tile_phase_kernel<false>, 1 tile_phase_kernel<true>,
// 2 tile_product_kernel, 3 any other kernel.
enum ProfKind : int { PK_LEAN = 0, PK_FAT = 1, PK_PROD = 2, PK_OTHER = 3, PK_COUNT = 4 };
struct ProfRec {
  hipEvent_t e0, e1;
  int slot;
  int kind;
  double flops;
};
struct Profiler {
  bool on = false;
  int calls = 0;   // evaluations whose launches are in recs (a graph counts once)
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<ProfRec> recs;
  hipEvent_t get() {
    if (used == pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
};
Profiler g_prof;

// Brackets one launch with events when profiling is on.
inline void prof_record(hipEvent_t e, hipStream_t s) { (void)hipEventRecord(e, s); }

struct ProfScope {
  ProfRec rec{nullptr, nullptr, 0, PK_OTHER, 0.0};
  hipStream_t s;
  ProfScope(int slot, double flops, hipStream_t st, int kind = PK_OTHER) : s(st) {
    if (!g_prof.on) return;
    rec.slot = slot;
    rec.kind = kind;
    rec.flops = flops;
    rec.e0 = g_prof.get();
    rec.e1 = g_prof.get();
    if (rec.e0 && rec.e1) prof_record(rec.e0, s);
  }
  ~ProfScope() {
    if (!g_prof.on || !rec.e0 || !rec.e1) return;
    prof_record(rec.e1, s);
    g_prof.recs.push_back(rec);
  }
};

inla_status run_phase(const Batch &B, int phase, int t, int p, hipStream_t s) {
  // (the batched V_t use the tile width of the step-by-step ones, so that
  // results do not depend on which of the two the workspace allowed)
  const bool big = B.big && phase_is_product_x(phase);
  long long total = 0;
  for (const auto &it : B.host) total += phase_tasks(it, phase, t, p, big);
  if (total > INT_MAX) return fail(INLA_ERR_ARG, "too many tile tasks in one launch");
  if (total == 0) return INLA_OK;
  double flops = 0.0;
  if (g_prof.on)
    for (const auto &it : B.host) flops += phase_flops(it, phase, t, p);
  // (the split-k scratch holds one b x b product per item: never the products
  // of every step)
  const bool every_step = phase == PH_SI_VU_B || phase == PH_SI_G_B;
  const int ks = (big && B.split && total < kSplitTiles && !every_step) ? kSplitK : 1;
  const bool prod = phase_is_product_x(phase) && (big || small_variant() > 0);
  ProfScope ps(phase, flops, s, prod ? PK_PROD : (phase_is_fat(phase) ? PK_FAT : PK_LEAN));
  HIP_TRY(launch_tile_phase(B.dev, (int)B.host.size(), (int)total, phase, -1, t, p, big, s, ks));
  return INLA_OK;
}

// Side stream (default priority) for phases that run beside another launch.
hipStream_t g_side = nullptr;
hipEvent_t g_fork = nullptr, g_join = nullptr;
// A second side stream (default priority) for the mode solve beside the
// selected inversion, with events of its own: the selected inversion forks to
// g_side itself.
hipStream_t g_solve = nullptr;
hipEvent_t g_solve_fork = nullptr, g_solve_join = nullptr;

// Runs phase pm on s and the independent phase ps of the same step on the side
// stream, joined back into s (in a captured graph: two parallel nodes).
inla_status run_beside(const Batch &B, int pm, int ps, int t, int p, hipStream_t s) {
  long long side = 0;
  for (const auto &it : B.host) side += phase_tasks(it, ps, t, p);
  if (side == 0) return run_phase(B, pm, t, p, s);
  if (!g_side) {
    HIP_TRY(hipStreamCreateWithFlags(&g_side, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&g_fork, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&g_join, hipEventDisableTiming));
  }
  HIP_TRY(hipEventRecord(g_fork, s));
  HIP_TRY(hipStreamWaitEvent(g_side, g_fork, 0));
  ST_TRY_INNER(run_phase(B, ps, t, p, g_side));
  ST_TRY_INNER(run_phase(B, pm, t, p, s));
  HIP_TRY(hipEventRecord(g_join, g_side));
  HIP_TRY(hipStreamWaitEvent(s, g_join, 0));
  return INLA_OK;
}

// Runs the b x b product phase px together with the independent phase pr of
// the same step: with 64-wide tiles in one launch (of the 64-tile kernel, or
// of the product kernel with pr's tasks first); with 128-wide tiles px on s
// and pr on a side stream joined back into s.
inla_status run_pair(const Batch &B, int px, int pr, int t, hipStream_t s) {
  if (!B.big && small_variant() == 0) {
    long long total = 0;
    double flops = 0.0;
    for (const auto &it : B.host) {
      total += phase_tasks(it, px, t, 0) + phase_tasks(it, pr, t, 0);
      if (g_prof.on) flops += phase_flops(it, px, t, 0) + phase_flops(it, pr, t, 0);
    }
    if (total > INT_MAX) return fail(INLA_ERR_ARG, "too many tile tasks in one launch");
    if (total == 0) return INLA_OK;
    ProfScope ps(px, flops, s, PK_LEAN);
    HIP_TRY(launch_tile_phase(B.dev, (int)B.host.size(), (int)total, px, pr, t, 0, false, s));
    return INLA_OK;
  }
  long long rem = 0;
  for (const auto &it : B.host) rem += phase_tasks(it, pr, t, 0);
  if (rem == 0) return run_phase(B, px, t, 0, s);
  if (!B.big) {
    // one launch of the product kernel: the side phase's tasks first, then the
    // tiles (with 128-wide tiles the side phase is larger, up to b^2 of copies
    // per item, and is better beside the launch than ahead of its tiles)
    long long tx = 0;
    for (const auto &it : B.host) tx += phase_tasks(it, px, t, 0);
    if (tx + rem + 8 > INT_MAX) return fail(INLA_ERR_ARG, "too many tile tasks in one launch");
    double flops = 0.0;
    if (g_prof.on)
      for (const auto &it : B.host) flops += phase_flops(it, px, t, 0) + phase_flops(it, pr, t, 0);
    ProfScope ps(px, flops, s, PK_PROD);
    HIP_TRY(launch_tile_phase(B.dev, (int)B.host.size(), (int)(tx + rem), px, pr, t, 0, B.big, s, 1,
                              (int)rem));
    return INLA_OK;
  }
  if (!g_side) {
    HIP_TRY(hipStreamCreateWithFlags(&g_side, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&g_fork, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&g_join, hipEventDisableTiming));
  }
  HIP_TRY(hipEventRecord(g_fork, s));
  HIP_TRY(hipStreamWaitEvent(g_side, g_fork, 0));
  ST_TRY_INNER(run_phase(B, pr, t, 0, g_side));
  HIP_TRY(hipEventRecord(g_join, g_side));
  ST_TRY_INNER(run_phase(B, px, t, 0, s));
  HIP_TRY(hipStreamWaitEvent(s, g_join, 0));
  return INLA_OK;
}

#define ST_TRY(expr)                     \
  do {                                   \
    inla_status st_ = (expr);            \
    if (st_ != INLA_OK) return st_;      \
  } while (0)

// The matrices of a batch eliminated from both ends: one pair of chains each.
struct Twist {
  std::vector<TwistPair> host;
  TwistPair *dev = nullptr;
  int max_a = 0, max_b = 0;
  int n() const { return (int)host.size(); }
  bool middle_at(int t) const {
    for (const auto &p : host)
      if (p.m == t) return true;
    return false;
  }
};
const Twist kNoTwist;

// Block Cholesky of the batch.  C holds the chains (a whole matrix is one
// chain; a matrix eliminated from both ends is two), F the whole matrices,
// which factor the arrow block once both chains have added their updates.
inla_status run_factor(const Batch &C, const Batch &F, const Twist &tw, hipStream_t s) {
  if (tw.n()) HIP_TRY(launch_twist_arrow(tw.dev, tw.n(), tw.max_a, 0, s));
  for (int t = 0; t < C.max_nt; ++t) {
    ST_TRY(run_phase(C, PH_DIAG0, t, 0, s));
    int mp = 0;
    for (const auto &it : C.host)
      if (t < it.nrun) mp = std::max(mp, it.nP);
    // Few tiles per step: one launch of the Cholesky-capable kernel per step (its
    // latency is the cost).  Many: the lean kernel for the step and the next
    // diagonal tile beside it.
    long long tiles2 = 0;
    for (const auto &it : C.host)
      if (t < it.nrun) tiles2 += (long long)it.nP * it.nP;
    const int fo = step_fused_override();
    const bool fused = fo < 0 ? tiles2 < kStepFusedTiles : fo == 1;
    for (int p = 0; p < mp; ++p) {
      if (fused) ST_TRY(run_phase(C, PH_STEPF, t, p, s));
      else ST_TRY(run_beside(C, PH_STEP, PH_DIAGC, t, p, s));
    }
    ST_TRY(run_pair(C, PH_OFFDIAG_X, PH_OFFDIAG, t, s));
    ST_TRY(run_pair(C, PH_SCHUR_X, PH_SCHUR, t, s));
  }
  if (tw.n()) HIP_TRY(launch_twist_arrow(tw.dev, tw.n(), tw.max_a, 1, s));
  ST_TRY(run_phase(F, PH_ARROW, 0, 0, s));
  return INLA_OK;
}

// Selected inversion: the arrow block by the whole matrices (F), then the
// block recursion down every chain (C); a backward chain starts from the
// middle block's Sigma, handed over once the forward chain has formed it.
inla_status run_selinv(const Batch &C, const Batch &F, const Twist &tw, bool traces, hipStream_t s) {
  ST_TRY(run_phase(F, PH_SI_INIT, 0, 0, s));
  if (traces) HIP_TRY(launch_trace_step(F.dev, (int)F.host.size(), -1, s));
  const int n = (int)C.host.size();
  if (C.vb) {
    // V_t, U_t and the first term of Sigma_D[t] need only the factor: every
    // step's at once, paired as the step-by-step phases are (so that each is
    // formed by the same code)
    ST_TRY(run_pair(C, PH_SI_VU_B, PH_SI_U_B, 0, s));
    ST_TRY(run_phase(C, PH_SI_G_B, 0, 0, s));
  }
  for (int t = C.max_nt - 1; t >= 0; --t) {
    if (!C.vb) ST_TRY(run_pair(C, PH_SI_VU_X, PH_SI_VU, t, s));
    ST_TRY(run_pair(C, PH_SI_SR_X, PH_SI_SR, t, s));
    ST_TRY(run_phase(C, PH_SI_SD_X, t, 0, s));
    if (traces) {
      ProfScope ps(PS_TRACE, 0.0, s);
      HIP_TRY(launch_trace_step(C.dev, n, t, s));
    }
    if (tw.middle_at(t)) HIP_TRY(launch_twist_middle(tw.dev, tw.n(), tw.max_b, tw.max_a, t, s));
  }
  return INLA_OK;
}

// Forward and backward substitution: the time blocks chain by chain (C, with
// per-chain vectors and scratch), the arrow block by the whole matrices (F).
inla_status run_solve(const Batch &C, const Batch &F, double *const *xs_c, double *const *tmps_c,
                      double *const *xs_f, double *const *tmps_f, hipStream_t s) {
  const int n = (int)C.host.size(), nf = (int)F.host.size();
  for (int t = 0; t < C.max_nt; ++t) {
    {
      ProfScope ps(PS_SOLVE, 0.0, s);
      HIP_TRY(launch_solve_stage(C.dev, n, C.max_b, C.max_a, t, SV_F1, xs_c, tmps_c, s));
    }
    {
      ProfScope ps(PS_SOLVE, 0.0, s);
      HIP_TRY(launch_solve_stage(C.dev, n, C.max_b, C.max_a, t, SV_F2, xs_c, tmps_c, s));
    }
  }
  if (F.max_a > 0) {
    HIP_TRY(launch_solve_stage(F.dev, nf, F.max_b, F.max_a, 0, SV_FA1, xs_f, tmps_f, s));
    HIP_TRY(launch_solve_stage(F.dev, nf, F.max_b, F.max_a, 0, SV_FA2, xs_f, tmps_f, s));
    HIP_TRY(launch_solve_stage(F.dev, nf, F.max_b, F.max_a, 0, SV_BA, xs_f, tmps_f, s));
  }
  for (int t = C.max_nt - 1; t >= 0; --t) {
    {
      ProfScope ps(PS_SOLVE, 0.0, s);
      HIP_TRY(launch_solve_stage(C.dev, n, C.max_b, C.max_a, t, SV_B1, xs_c, tmps_c, s));
    }
    {
      ProfScope ps(PS_SOLVE, 0.0, s);
      HIP_TRY(launch_solve_stage(C.dev, n, C.max_b, C.max_a, t, SV_B2, xs_c, tmps_c, s));
    }
  }
  return INLA_OK;
}

inla_status check_bta(const inla_bta *q, const char *what) {
  if (!q) return fail(INLA_ERR_ARG, std::string(what) + " is NULL");
  if (q->b < 1 || q->nt < 1 || q->a < 0 || q->a > kMaxArrow)
    return fail(INLA_ERR_ARG, std::string(what) + ": need b >= 1, nt >= 1, 0 <= a <= 64");
  if (!q->D || (q->nt > 1 && !q->S) || (q->a > 0 && (!q->R || !q->T)))
    return fail(INLA_ERR_ARG, std::string(what) + ": missing block pointer");
  if ((long long)q->b * q->b > (1LL << 40))
    return fail(INLA_ERR_ARG, std::string(what) + ": block too large");
  return INLA_OK;
}

ItemDev item_from_bta(const inla_bta &q) {
  ItemDev it;
  std::memset(&it, 0, sizeof(it));
  it.b = q.b; it.nt = q.nt; it.a = q.a; it.nP = ntile(q.b);
  it.ntf = q.nt; it.trev = 0; it.nrun = q.nt; it.own_arrow = 1;
  it.sbw = q.b;   // a caller's coupling blocks are taken as dense
  it.D = q.D; it.S = q.S; it.R = q.R; it.T = q.T;
  return it;
}

// Workspace of one item's factorization.
void layout_factor_ws(Layout &L, ItemDev &it) {
  const size_t bb = (size_t)it.b * it.b;
  L.add(&it.W1, bb);
  L.add(&it.W2, bb);
  L.add(&it.W3, std::max<size_t>((size_t)it.a * it.b, 1));
  L.add(&it.Mp, 2 * (size_t)kTile * kTile);
  L.add(&it.ldpart, (size_t)it.nt * it.nP + 1);
  L.add(&it.info, 1);
}

// Workspace of one item's selected inversion when Sigma is streamed.
void layout_selinv_ws(Layout &L, ItemDev &it) {
  const size_t bb = (size_t)it.b * it.b;
  L.add(&it.SD, 2 * bb);
  L.add(&it.SR, std::max<size_t>(2 * (size_t)it.a * it.b, 1));
  L.add(&it.ST, std::max<size_t>((size_t)it.a * it.a, 1));
}

size_t bta_doubles(int b, int nt, int a) {
  return (size_t)(2 * nt - 1) * b * b + (size_t)nt * a * b + (size_t)a * a;
}

// The launch sequence of one batched evaluation, captured once per call
// signature and replayed.  Inputs and outputs pass through library buffers so
// the captured graph only ever touches library memory.
struct EvalGraph {
  bool valid = false;
  GraphKey key;
  hipGraphExec_t exec = nullptr;
  double *th = nullptr, *f = nullptr, *g = nullptr, *mu_buf = nullptr, *var_buf = nullptr;
  int *st = nullptr;
};
EvalGraph g_graph;
hipStream_t g_cap = nullptr;

bool graphs_enabled() {
  const char *e = getenv("INLA_GRAPH");
  return !(e && e[0] == '0');
}

void drop_graph() {
  if (g_graph.exec) (void)hipGraphExecDestroy(g_graph.exec);
  g_graph = EvalGraph();
}

void drop_graph_of_model(uint64_t id) {
  if (g_graph.valid && key_uses_model(g_graph.key, id)) drop_graph();
}

// ---------------------------------------------------------------------------
// workspace of the allocation-free factorization: one fixed device array per
// GPU, held from the first call on that GPU until the process ends
// ---------------------------------------------------------------------------
constexpr size_t kNoAllocScratchBytes = INLA_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];
constexpr int kMaxDevices = 64;
// Device address of `scratch` on each GPU (host code must never pass the
// array's name itself to a kernel: on the host it is only a stand-in).
char *g_scratch_ptr[kMaxDevices] = {};

inla_status ensure_streams();

// Set-up on the first call on the current device: the array's device address
// and the library's side streams (so that later calls create nothing).
// Called with g_mutex held.
inla_status noalloc_scratch(char **out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(INLA_ERR_STATE, "device index out of range");
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(INLA_ERR_STATE, "no device address for the fixed workspace");
    ST_TRY_INNER(ensure_streams());
    g_scratch_ptr[dev] = static_cast<char *>(p);
  }
  *out = g_scratch_ptr[dev];
  return INLA_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// model
// ---------------------------------------------------------------------------
struct inla_model {
  ModelDev host;      // field values with device pointers
  ModelDev *dev = nullptr;
  void *mem = nullptr;
  int device = 0;
  long long n = 0, m = 0;
  uint64_t id = 0;    // unique over the process lifetime (captured graphs key on it)
  bool counts = false;       // every y_i is a non-negative integer (a count likelihood may use it)
  double log_y_fact = 0.0;   // sum_i log(y_i!) when counts
};

namespace inla {
const ModelDev *model_device(const inla_model *m) { return m->dev; }
const ModelDev &model_host_desc(const inla_model *m) { return m->host; }
bool model_counts(const inla_model *m, double *log_y_fact) {
  if (log_y_fact) *log_y_fact = m->log_y_fact;
  return m->counts;
}
}  // namespace inla

namespace {

std::atomic<uint64_t> g_next_model_id{1};

struct HostModel {
  int N, nt, a, b;
  int sbw = 0;   // half-bandwidth of Q_s (the largest |i - s| of a nonzero entry)
  std::vector<int> colptr, rowidx, colidx;
  std::vector<double> pdelta, pg1, pg2, AtA, ZtA, ZtZ, Aty;
};

inla_status build_host_model(const inla_model_desc &d, HostModel &hm) {
  const int N = d.N, nt = d.nt, a = d.nb;
  const int b = N * N;
  const long long nst = (long long)b * nt, n = nst + a;
  hm.N = N; hm.nt = nt; hm.a = a; hm.b = b;
  // Q_s pattern: all nodes within grid distance |dx| + |dy| <= 2 of each node
  // (the reach of G^2), plus any extra pair that A^T A couples.
  std::vector<std::vector<int>> rows(b);
  auto grid_ok = [&](int x, int y) { return x >= 0 && x < N && y >= 0 && y < N; };
  for (int sy = 0; sy < N; ++sy)
    for (int sx = 0; sx < N; ++sx) {
      auto &r = rows[sy * N + sx];
      for (int dy = -2; dy <= 2; ++dy)
        for (int dx = -2; dx <= 2; ++dx)
          if (std::abs(dx) + std::abs(dy) <= 2 && grid_ok(sx + dx, sy + dy))
            r.push_back((sy + dy) * N + (sx + dx));
    }
  // validate A and collect extra couplings
  for (long long j = 0; j < d.m; ++j) {
    const long long e0 = d.A_rowptr[j], e1 = d.A_rowptr[j + 1];
    if (e1 < e0) return fail(INLA_ERR_ARG, "A_rowptr is not non-decreasing");
    int tj = -1;
    for (long long e = e0; e < e1; ++e) {
      const long long c = d.A_col[e];
      if (c < 0 || c >= n) return fail(INLA_ERR_ARG, "A column index out of range");
      if (c < nst) {
        const int t = (int)(c / b);
        if (tj >= 0 && t != tj) return fail(INLA_ERR_ARG, "an observation couples two time blocks");
        tj = t;
      }
    }
    for (long long e = e0; e < e1; ++e) {
      const long long ce = d.A_col[e];
      if (ce >= nst) continue;
      const int se = (int)(ce % b);
      for (long long f = e0; f < e1; ++f) {
        const long long cf = d.A_col[f];
        if (cf >= nst) continue;
        const int sf = (int)(cf % b);
        const int ex = se % N, ey = se / N, fx = sf % N, fy = sf / N;
        if (std::abs(ex - fx) + std::abs(ey - fy) > 2) rows[sf].push_back(se);
      }
    }
  }
  hm.colptr.assign(b + 1, 0);
  for (int s = 0; s < b; ++s) {
    auto &r = rows[s];
    std::sort(r.begin(), r.end());
    r.erase(std::unique(r.begin(), r.end()), r.end());
    hm.colptr[s + 1] = hm.colptr[s] + (int)r.size();
  }
  const int nnz = hm.colptr[b];
  hm.rowidx.resize(nnz);
  hm.colidx.resize(nnz);
  for (int s = 0; s < b; ++s)
    for (size_t k = 0; k < rows[s].size(); ++k) {
      hm.rowidx[hm.colptr[s] + k] = rows[s][k];
      hm.colidx[hm.colptr[s] + k] = s;
    }
  auto find = [&](int i, int s) -> int {
    const int *lo = hm.rowidx.data() + hm.colptr[s], *hi = hm.rowidx.data() + hm.colptr[s + 1];
    const int *p = std::lower_bound(lo, hi, i);
    return (p != hi && *p == i) ? (int)(p - hm.rowidx.data()) : -1;
  };
  // G (4-neighbour Neumann Laplacian) and G^2 on the pattern
  auto Gval = [&](int i, int s) -> double {
    const int ix = i % N, iy = i / N, sx = s % N, sy = s / N;
    if (i == s) {
      int deg = 0;
      if (sx > 0) ++deg;
      if (sx < N - 1) ++deg;
      if (sy > 0) ++deg;
      if (sy < N - 1) ++deg;
      return deg;
    }
    return (std::abs(ix - sx) + std::abs(iy - sy) == 1) ? -1.0 : 0.0;
  };
  hm.pdelta.assign(nnz, 0.0);
  hm.pg1.assign(nnz, 0.0);
  hm.pg2.assign(nnz, 0.0);
  for (int s = 0; s < b; ++s) {
    const int sx = s % N, sy = s / N;
    for (int e = hm.colptr[s]; e < hm.colptr[s + 1]; ++e) {
      const int i = hm.rowidx[e];
      hm.pdelta[e] = (i == s) ? 1.0 : 0.0;
      hm.pg1[e] = Gval(i, s);
      // (G^2)(i,s) = sum_u G(i,u) G(u,s), u over s and its neighbours
      double g2 = 0.0;
      const int us[5][2] = {{0, 0}, {-1, 0}, {1, 0}, {0, -1}, {0, 1}};
      for (auto &du : us) {
        const int ux = sx + du[0], uy = sy + du[1];
        if (!grid_ok(ux, uy)) continue;
        const int u = uy * N + ux;
        g2 += Gval(i, u) * Gval(u, s);
      }
      hm.pg2[e] = g2;
      if (hm.pdelta[e] != 0.0 || hm.pg1[e] != 0.0 || g2 != 0.0) hm.sbw = std::max(hm.sbw, std::abs(i - s));
    }
  }
  // A^T A per time block, Z^T A_t, Z^T Z, A^T y (row order: deterministic sums)
  hm.AtA.assign((size_t)nt * nnz, 0.0);
  hm.ZtA.assign((size_t)nt * a * b, 0.0);
  hm.ZtZ.assign((size_t)a * a, 0.0);
  hm.Aty.assign((size_t)n, 0.0);
  for (long long j = 0; j < d.m; ++j) {
    const long long e0 = d.A_rowptr[j], e1 = d.A_rowptr[j + 1];
    const double yj = d.y[j];
    for (long long e = e0; e < e1; ++e) hm.Aty[d.A_col[e]] += d.A_val[e] * yj;
    for (long long e = e0; e < e1; ++e) {
      const long long ce = d.A_col[e];
      const double ve = d.A_val[e];
      for (long long f = e0; f < e1; ++f) {
        const long long cf = d.A_col[f];
        const double vf = d.A_val[f];
        if (ce < nst && cf < nst) {
          const int t = (int)(ce / b);
          const int k = find((int)(ce % b), (int)(cf % b));
          hm.AtA[(size_t)t * nnz + k] += ve * vf;
        } else if (ce >= nst && cf < nst) {
          const int t = (int)(cf / b);
          hm.ZtA[(size_t)t * a * b + (size_t)(cf % b) * a + (ce - nst)] += ve * vf;
        } else if (ce >= nst && cf >= nst) {
          hm.ZtZ[(size_t)(ce - nst) + (size_t)(cf - nst) * a] += ve * vf;
        }
      }
    }
  }
  return INLA_OK;
}

}  // namespace

extern "C" {

const char *inla_status_string(inla_status s) {
  switch (s) {
    case INLA_OK: return "ok";
    case INLA_ERR_ARG: return "invalid argument";
    case INLA_ERR_NOT_SPD: return "matrix not positive definite";
    case INLA_ERR_BUDGET: return "item exceeds the HBM budget";
    case INLA_ERR_HIP: return "HIP runtime error";
    case INLA_ERR_NOMEM: return "out of memory";
    case INLA_ERR_STATE: return "library not usable";
  }
  return "unknown status";
}

const char *inla_last_error(void) { return g_last_error.c_str(); }

#ifndef INLA_SOURCE_HASH
#define INLA_SOURCE_HASH "unknown"
#endif
const char *inla_build_id(void) { return INLA_SOURCE_HASH; }

inla_status inla_model_create(const inla_model_desc *desc, void *hip_stream, inla_model **out) {
  g_last_error.clear();
  if (!desc || !out) return fail(INLA_ERR_ARG, "desc and out must be non-NULL");
  *out = nullptr;
  const inla_model_desc &d = *desc;
  if (d.N < 1 || d.nt < 1 || d.nb < 0 || d.nb > kMaxArrow)
    return fail(INLA_ERR_ARG, "need N >= 1, nt >= 1, 0 <= nb <= 64");
  if (!(d.h > 0.0) || !(d.beta_prior_prec > 0.0))
    return fail(INLA_ERR_ARG, "need h > 0 and beta_prior_prec > 0");
  if (d.m < 1 || !d.A_rowptr || !d.A_col || !d.A_val || !d.y || !d.theta_prior_mean ||
      !d.theta_prior_prec)
    return fail(INLA_ERR_ARG, "missing observation data or hyperprior");
  if ((long long)d.N * d.N > 65536) return fail(INLA_ERR_ARG, "N*N above 65536 not supported");
  for (int k = 0; k < 4; ++k)
    if (!(d.theta_prior_prec[k] > 0.0)) return fail(INLA_ERR_ARG, "hyperprior precision must be > 0");
  HostModel hm;
  ST_TRY(build_host_model(d, hm));
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  inla_model *M = new inla_model();
  HIP_TRY(hipGetDevice(&M->device));
  const int b = hm.b, nt = hm.nt, a = hm.a;
  const long long n = (long long)b * nt + a;
  const long long nnzA = d.A_rowptr[d.m];
  M->n = n;
  M->m = d.m;
  ModelDev &h = M->host;
  std::memset(&h, 0, sizeof(h));
  h.N = d.N; h.nt = nt; h.a = a; h.b = b; h.m = d.m; h.n = n; h.h = d.h;
  h.beta_prec = d.beta_prior_prec;
  for (int k = 0; k < 4; ++k) {
    h.prior_mean[k] = d.theta_prior_mean[k];
    h.prior_prec[k] = d.theta_prior_prec[k];
  }
  h.nnz = hm.colptr[b];
  h.sbw = std::min(hm.sbw, b);
  Layout L;
  int *colptr, *rowidx, *colidx, *A_col;
  double *pdelta, *pg1, *pg2, *AtA, *ZtA, *ZtZ, *Aty, *A_val, *y;
  long long *A_rowptr;
  ModelDev *mdev;
  L.add(&mdev, 1);
  L.add(&colptr, hm.colptr.size());
  L.add(&rowidx, hm.rowidx.size());
  L.add(&colidx, hm.colidx.size());
  L.add(&pdelta, hm.pdelta.size());
  L.add(&pg1, hm.pg1.size());
  L.add(&pg2, hm.pg2.size());
  L.add(&AtA, hm.AtA.size());
  L.add(&ZtA, std::max<size_t>(hm.ZtA.size(), 1));
  L.add(&ZtZ, std::max<size_t>(hm.ZtZ.size(), 1));
  L.add(&Aty, hm.Aty.size());
  L.add(&A_rowptr, (size_t)d.m + 1);
  L.add(&A_col, (size_t)nnzA);
  L.add(&A_val, (size_t)nnzA);
  L.add(&y, (size_t)d.m);
  // A by columns and the dense fixed-effect columns
  std::vector<long long> cptr((size_t)n + 1, 0);
  for (long long e = 0; e < nnzA; ++e) ++cptr[(size_t)d.A_col[e] + 1];
  for (long long j = 0; j < n; ++j) cptr[j + 1] += cptr[j];
  std::vector<int> crow((size_t)nnzA);
  std::vector<double> cval((size_t)nnzA);
  std::vector<long long> cfill(cptr.begin(), cptr.end() - 1);
  std::vector<double> Zd((size_t)d.m * a, 0.0);
  for (long long i = 0; i < d.m; ++i)
    for (long long e = d.A_rowptr[i]; e < d.A_rowptr[i + 1]; ++e) {
      const int c = d.A_col[e];
      long long &q = cfill[c];
      if (q > cptr[c] && crow[q - 1] == (int)i) {
        cval[q - 1] += d.A_val[e];   // a repeated column within the row
      } else {
        crow[q] = (int)i;
        cval[q] = d.A_val[e];
        ++q;
      }
      if (c >= (long long)b * nt) Zd[(size_t)i * a + (c - (long long)b * nt)] += d.A_val[e];
    }
  // compact the columns (repeats leave gaps)
  {
    long long w = 0;
    for (long long j = 0; j < n; ++j) {
      const long long r0 = cptr[j], r1 = cfill[j];
      cptr[j] = w;
      for (long long q = r0; q < r1; ++q, ++w) {
        crow[w] = crow[q];
        cval[w] = cval[q];
      }
    }
    cptr[n] = w;
  }
  const long long nnzC = cptr[n];
  long long *Ac_ptr;
  int *Ac_row;
  double *Ac_val, *Zdd;
  L.add(&Ac_ptr, (size_t)n + 1);
  L.add(&Ac_row, (size_t)std::max<long long>(nnzC, 1));
  L.add(&Ac_val, (size_t)std::max<long long>(nnzC, 1));
  L.add(&Zdd, std::max<size_t>(Zd.size(), 1));
  M->counts = true;
  for (long long i = 0; i < d.m; ++i) {
    const double yi = d.y[i];
    if (!(std::isfinite(yi) && yi >= 0.0 && yi == std::floor(yi))) {
      M->counts = false;
      break;
    }
    M->log_y_fact += std::lgamma(yi + 1.0);
  }
  if (!M->counts) M->log_y_fact = 0.0;
  if (hipMalloc(&M->mem, L.total) != hipSuccess) {
    (void)hipGetLastError();
    delete M;
    return fail(INLA_ERR_NOMEM, "model allocation failed");
  }
  size_t off = 0;
  for (auto &r : L.reqs) {
    *r.slot = static_cast<char *>(M->mem) + off;
    off += align_up(std::max<size_t>(r.bytes, 1));
  }
  auto put = [&](void *dst, const void *src, size_t bytes) -> hipError_t {
    if (!bytes) return hipSuccess;
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
  };
  h.colptr = colptr; h.rowidx = rowidx; h.colidx = colidx; h.pdelta = pdelta; h.pg1 = pg1;
  h.pg2 = pg2; h.AtA = AtA; h.ZtA = ZtA; h.ZtZ = ZtZ; h.Aty = Aty; h.A_rowptr = A_rowptr;
  h.A_col = A_col; h.A_val = A_val; h.y = y;
  h.Ac_ptr = Ac_ptr; h.Ac_row = Ac_row; h.Ac_val = Ac_val; h.Zd = Zdd;
  hipError_t e = hipSuccess;
  if (!e) e = put(colptr, hm.colptr.data(), hm.colptr.size() * sizeof(int));
  if (!e) e = put(rowidx, hm.rowidx.data(), hm.rowidx.size() * sizeof(int));
  if (!e) e = put(colidx, hm.colidx.data(), hm.colidx.size() * sizeof(int));
  if (!e) e = put(pdelta, hm.pdelta.data(), hm.pdelta.size() * sizeof(double));
  if (!e) e = put(pg1, hm.pg1.data(), hm.pg1.size() * sizeof(double));
  if (!e) e = put(pg2, hm.pg2.data(), hm.pg2.size() * sizeof(double));
  if (!e) e = put(AtA, hm.AtA.data(), hm.AtA.size() * sizeof(double));
  if (!e) e = put(ZtA, hm.ZtA.data(), hm.ZtA.size() * sizeof(double));
  if (!e) e = put(ZtZ, hm.ZtZ.data(), hm.ZtZ.size() * sizeof(double));
  if (!e) e = put(Aty, hm.Aty.data(), hm.Aty.size() * sizeof(double));
  if (!e) e = put(A_rowptr, d.A_rowptr, ((size_t)d.m + 1) * sizeof(long long));
  if (!e) e = put(A_col, d.A_col, (size_t)nnzA * sizeof(int));
  if (!e) e = put(A_val, d.A_val, (size_t)nnzA * sizeof(double));
  if (!e) e = put(y, d.y, (size_t)d.m * sizeof(double));
  if (!e) e = put(Ac_ptr, cptr.data(), cptr.size() * sizeof(long long));
  if (!e) e = put(Ac_row, crow.data(), (size_t)nnzC * sizeof(int));
  if (!e) e = put(Ac_val, cval.data(), (size_t)nnzC * sizeof(double));
  if (!e) e = put(Zdd, Zd.data(), Zd.size() * sizeof(double));
  if (!e) e = put(mdev, &h, sizeof(ModelDev));
  if (!e) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    (void)hipFree(M->mem);
    delete M;
    return fail(INLA_ERR_HIP, std::string("model upload: ") + hipGetErrorString(e));
  }
  M->dev = mdev;
  M->id = g_next_model_id.fetch_add(1);
  *out = M;
  return INLA_OK;
}

void inla_model_destroy(inla_model *model) {
  if (!model) return;
  {
    std::lock_guard<std::mutex> lk(g_mutex);
    if (g_arena.last) (void)hipEventSynchronize(g_arena.last);
    // a captured graph that reads this model's data must never run again
    drop_graph_of_model(model->id);
  }
  if (model->mem) (void)hipFree(model->mem);
  delete model;
}

inla_status inla_model_shape(const inla_model *model, int32_t *b, int32_t *nt, int32_t *a,
                             int64_t *n, int64_t *m) {
  if (!model) return fail(INLA_ERR_ARG, "model is NULL");
  if (b) *b = model->host.b;
  if (nt) *nt = model->host.nt;
  if (a) *a = model->host.a;
  if (n) *n = model->n;
  if (m) *m = model->m;
  return INLA_OK;
}

inla_status inla_assemble(const inla_model *model, const double *theta_dev, int32_t which,
                          inla_bta *out, double *rhs_dev, void *hip_stream) {
  g_last_error.clear();
  if (!model || !theta_dev) return fail(INLA_ERR_ARG, "model and theta must be non-NULL");
  if (which != 0 && which != 1) return fail(INLA_ERR_ARG, "which must be 0 or 1");
  ST_TRY(check_bta(out, "out"));
  const ModelDev &h = model->host;
  if (out->b != h.b || out->nt != h.nt || out->a != h.a)
    return fail(INLA_ERR_ARG, "out shape does not match the model");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  HIP_TRY(launch_assemble(model->dev, h.b, h.nt, h.a, theta_dev, which, out->D, out->S, out->R,
                          out->T, which ? rhs_dev : nullptr, s));
  return INLA_OK;
}

inla_status inla_factor_logdet(inla_bta *QL, double *logdet_dev, int32_t *info_dev,
                               void *hip_stream) {
  g_last_error.clear();
  ST_TRY(check_bta(QL, "QL"));
  std::lock_guard<std::mutex> lk(g_mutex);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  Batch B;
  B.host.push_back(item_from_bta(*QL));
  Layout L;
  layout_factor_ws(L, B.host[0]);
  L.add(&B.dev, 1);
  double *ld_tmp;
  int *info_tmp;
  L.add(&ld_tmp, 1);
  L.add(&info_tmp, 1);
  ST_TRY(arena_bind(L, s));
  B.finalize();
  HIP_TRY(launch_fill_int(B.host[0].info, 1, kInfoNone, s));
  ST_TRY(upload(B.dev, B.host, s));
  ST_TRY(run_factor(B, B, kNoTwist, s));
  HIP_TRY(launch_logdet_finish(B.dev, 1, logdet_dev ? logdet_dev : ld_tmp,
                               info_dev ? info_dev : info_tmp, s));
  return arena_done(s);
}

inla_status inla_factor_logdet_noalloc(inla_bta *QL, double *logdet_dev, int32_t *info_dev,
                                       void *hip_stream) {
  g_last_error.clear();
  ST_TRY(check_bta(QL, "QL"));
  std::lock_guard<std::mutex> lk(g_mutex);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  char *base = nullptr;
  ST_TRY(noalloc_scratch(&base));
  Batch B;
  B.host.push_back(item_from_bta(*QL));
  Layout L;
  layout_factor_ws(L, B.host[0]);
  L.add(&B.dev, 1);
  double *ld_tmp;
  int *info_tmp;
  L.add(&ld_tmp, 1);
  L.add(&info_tmp, 1);
  if (L.total > kNoAllocScratchBytes)
    return fail(INLA_ERR_BUDGET, "the factorization needs " + std::to_string(L.total) +
                                     " bytes of workspace, above the " +
                                     std::to_string(kNoAllocScratchBytes) +
                                     " bytes of inla_factor_logdet_noalloc");
  size_t off = 0;
  for (auto &r : L.reqs) {
    *r.slot = base + off;
    off += align_up(std::max<size_t>(r.bytes, 1));
  }
  B.finalize();
  // no event pool growth and no records: this entry point is never profiled
  const bool prof = g_prof.on;
  g_prof.on = false;
  auto body = [&]() -> inla_status {
    // the first failing pivot starts at "none"; the descriptor travels as a
    // kernel argument (nothing is staged in host memory)
    HIP_TRY(launch_fill_int(B.host[0].info, 1, kInfoNone, s));
    HIP_TRY(launch_put_item(B.host[0], B.dev, s));
    ST_TRY(run_factor(B, B, kNoTwist, s));
    HIP_TRY(launch_logdet_finish(B.dev, 1, logdet_dev ? logdet_dev : ld_tmp,
                                 info_dev ? info_dev : info_tmp, s));
    return INLA_OK;
  };
  const inla_status st = body();
  g_prof.on = prof;
  return st;
}

inla_status inla_solve(const inla_bta *L_, const double *rhs_dev, double *x_dev, int32_t nrhs,
                       void *hip_stream) {
  g_last_error.clear();
  ST_TRY(check_bta(L_, "L"));
  if (nrhs < 1 || !rhs_dev || !x_dev) return fail(INLA_ERR_ARG, "need nrhs >= 1 and vectors");
  std::lock_guard<std::mutex> lk(g_mutex);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const long long n = (long long)L_->b * L_->nt + L_->a;
  Batch B;
  for (int r = 0; r < nrhs; ++r) B.host.push_back(item_from_bta(*L_));
  B.finalize();
  Layout L;
  L.add(&B.dev, nrhs);
  double **xs, **tmps, *tmp;
  L.add(&xs, nrhs);
  L.add(&tmps, nrhs);
  const size_t tl = std::max(L_->b, std::max(L_->a, 1));
  L.add(&tmp, tl * nrhs);
  ST_TRY(arena_bind(L, s));
  if (x_dev != rhs_dev)
    HIP_TRY(hipMemcpyAsync(x_dev, rhs_dev, (size_t)n * nrhs * sizeof(double),
                           hipMemcpyDeviceToDevice, s));
  std::vector<double *> hx(nrhs), ht(nrhs);
  for (int r = 0; r < nrhs; ++r) {
    hx[r] = x_dev + (size_t)r * n;
    ht[r] = tmp + (size_t)r * tl;
  }
  ST_TRY(upload(B.dev, B.host, s));
  ST_TRY(upload(xs, hx, s));
  ST_TRY(upload(tmps, ht, s));
  ST_TRY(run_solve(B, B, xs, tmps, xs, tmps, s));
  return arena_done(s);
}

inla_status inla_selinv(const inla_bta *L_, inla_bta *sigma_or_null, double *diag_or_null,
                        void *hip_stream) {
  g_last_error.clear();
  ST_TRY(check_bta(L_, "L"));
  if (sigma_or_null) {
    ST_TRY(check_bta(sigma_or_null, "sigma"));
    if (sigma_or_null->b != L_->b || sigma_or_null->nt != L_->nt || sigma_or_null->a != L_->a)
      return fail(INLA_ERR_ARG, "sigma shape does not match L");
  }
  std::lock_guard<std::mutex> lk(g_mutex);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  Batch B;
  B.host.push_back(item_from_bta(*L_));
  ItemDev &it = B.host[0];
  Layout L;
  const size_t bb = (size_t)it.b * it.b;
  L.add(&it.W2, bb);
  L.add(&it.W3, std::max<size_t>((size_t)it.a * it.b, 1));
  L.add(&it.Mp, 2 * (size_t)kTile * kTile);
  if (sigma_or_null) {
    it.SD = sigma_or_null->D; it.sd_stride = (long long)bb;
    it.SS = sigma_or_null->S; it.ss_stride = (long long)bb;
    it.SR = sigma_or_null->R; it.sr_stride = (long long)it.a * it.b;
    it.ST = sigma_or_null->T;
  } else {
    layout_selinv_ws(L, it);
    L.add(&it.SS, bb);
  }
  it.diag = diag_or_null;
  L.add(&B.dev, 1);
  ST_TRY(arena_bind(L, s));
  B.finalize();
  ST_TRY(upload(B.dev, B.host, s));
  ST_TRY(run_selinv(B, B, kNoTwist, diag_or_null != nullptr, s));
  return arena_done(s);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batched f(theta) and gradient
// ---------------------------------------------------------------------------
namespace {

struct ThetaItemBufs {
  ItemDev P, C;        // the whole matrices
  ItemDev Pb, Cb;      // their backward chains (two-sided elimination)
  bool tw = false;     // the matrices are eliminated from both ends
  double *x = nullptr, *tmp = nullptr, *tmpb = nullptr, *term = nullptr;
  double *TBp = nullptr, *TBc = nullptr;   // arrow accumulators of the backward chains
};

// Whether a matrix of nt time blocks is eliminated from both ends: from four
// blocks on (two steps in each direction), unless INLA_TWIST=0 in the
// environment or the call keeps the selected inverse in caller storage.
bool twist_env() {
  const char *e = getenv("INLA_TWIST");
  return !(e && e[0] == '0');
}
bool twisted(const ModelDev &h, bool allowed) { return allowed && h.nt >= 4; }

// Device bytes one (model, theta) item needs: two BTA matrices with their
// workspaces, or one shared by Q_prior and Q_c when `seq` (the two are then
// processed one after the other); `vb`: the selected inversion keeps V_t and
// U_t of every step; `tw`: the matrices are eliminated from both ends (the
// backward chains have workspaces of their own).
size_t theta_item_bytes(const ModelDev &h, bool selinv, bool seq, bool split, bool vb, bool tw) {
  const size_t bb = (size_t)h.b * h.b, ab = (size_t)h.a * h.b;
  const int nP = ntile(h.b);
  size_t per = bta_doubles(h.b, h.nt, h.a) * 8 + (2 * bb + ab + 2 * kTile * kTile) * 8 +
               ((size_t)h.nt * nP + 1) * 8 + 5 * kAlign * 4;
  if (selinv) per += (2 * bb + 2 * ab + (size_t)h.a * h.a) * 8 + ((size_t)h.nt + 1) * kTraceBlocks * 32;
  if (selinv && vb) per += ((size_t)(2 * h.nt - 1) * bb + (size_t)h.nt * ab) * 8 + 3 * kAlign;
  if (split) per += (size_t)kSplitK * bb * 8 + kAlign;
  if (tw) {
    per += (2 * bb + ab + 2 * kTile * kTile + (size_t)h.a * h.a) * 8 + 5 * kAlign;
    if (split) per += (size_t)kSplitK * bb * 8 + kAlign;
    if (selinv) per += (2 * bb + 2 * ab) * 8 + 2 * kAlign;
  }
  return (seq ? 1 : 2) * per + ((size_t)h.n + 2 * std::max(h.b, h.a) + kTermBlocks * 4) * 8 + 4096;
}

inla_status ensure_streams() {
  if (!g_side) {
    HIP_TRY(hipStreamCreateWithFlags(&g_side, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&g_fork, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&g_join, hipEventDisableTiming));
  }
  if (!g_cap) HIP_TRY(hipStreamCreateWithFlags(&g_cap, hipStreamNonBlocking));
  if (!g_solve) {
    HIP_TRY(hipStreamCreateWithFlags(&g_solve, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&g_solve_fork, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&g_solve_join, hipEventDisableTiming));
  }
  return INLA_OK;
}

// Copies a replayed graph's outputs to the caller; ntot is this call's total
// length of mu / var (equal to the graph's: it is part of the key).
inla_status copy_outputs(const EvalGraph &G, int n, long long ntot, double *f_dev, double *grad_dev,
                         double *mu_out, double *var_out, int32_t *status_dev, hipStream_t s) {
  const auto D2D = hipMemcpyDeviceToDevice;
  HIP_TRY(hipMemcpyAsync(f_dev, G.f, (size_t)n * 8, D2D, s));
  if (grad_dev) HIP_TRY(hipMemcpyAsync(grad_dev, G.g, (size_t)n * 32, D2D, s));
  if (status_dev) HIP_TRY(hipMemcpyAsync(status_dev, G.st, (size_t)n * 4, D2D, s));
  if (G.key.ntot != ntot) return fail(INLA_ERR_STATE, "internal: replayed graph has another output size");
  if (mu_out) HIP_TRY(hipMemcpyAsync(mu_out, G.mu_buf, (size_t)ntot * 8, D2D, s));
  if (var_out) HIP_TRY(hipMemcpyAsync(var_out, G.var_buf, (size_t)ntot * 8, D2D, s));
  return INLA_OK;
}

// Layout choices of one batched evaluation and the bytes each item needs.
struct EvalPlan {
  bool grad = false, need_selinv = false, twist_ok = false;
  bool seq = false, split = false, vb = false;
  int waves = 0;
  std::vector<size_t> bytes;   // per item
  double all = 0.0;            // summed over the items
};

// HBM admission: the layout with the fewest waves whose storage fits the
// budget.  `seq_mode`: 2 never, 1 always, 0 when the two-matrix layout needs
// more admission waves than the one-matrix layout.
inla_status plan_eval(const inla_model *const *models, int32_t n_items, bool grad, bool need_selinv,
                      double budget, int seq_mode, bool twist_ok, EvalPlan &P) {
  P.grad = grad;
  P.need_selinv = need_selinv;
  P.twist_ok = twist_ok;
  // split-k scratch when the whole call has few 128-wide tiles per launch
  long long nb2 = 0;
  for (int i = 0; i < n_items; ++i) nb2 += 2LL * nbig(models[i]->host.b) * nbig(models[i]->host.b);
  const bool split_wanted = nb2 < kSplitTiles && tile_request() == 128;
  // V_t and U_t of every step up front when the step-by-step launches of the
  // selected inversion would have few tiles
  long long nv = 0;
  for (int i = 0; i < n_items; ++i) nv += 2LL * ntile(models[i]->host.b) * ntile(models[i]->host.b);
  const bool vb_wanted = need_selinv && nv < kVBatchTiles && si_batch_allowed();
  auto waves_for = [&](bool seq, bool split, bool vb, std::vector<size_t> &bytes,
                       double &all) -> int {
    bytes.assign(n_items, 0);
    all = 0.0;
    int waves = 0;
    double acc = budget + 1.0;
    for (int i = 0; i < n_items; ++i) {
      bytes[i] = theta_item_bytes(models[i]->host, need_selinv, seq, split, vb,
                                  twisted(models[i]->host, twist_ok));
      all += (double)bytes[i];
      if ((double)bytes[i] > budget) return INT_MAX;
      if (acc + (double)bytes[i] > budget) {
        ++waves;
        acc = 0.0;
      }
      acc += (double)bytes[i];
    }
    return waves;
  };
  // layouts in order of preference; the first with the fewest waves wins
  struct Cand { bool seq, split, vb; };
  std::vector<Cand> cands;
  for (int sq = 0; sq < 2; ++sq) {
    const bool seq_c = sq == 1;
    if ((seq_mode == 1 && !seq_c) || (seq_mode == 2 && seq_c)) continue;
    for (int v = 0; v < 2; ++v) {
      const bool vb_c = v == 0;
      if (vb_c && !vb_wanted) continue;
      if (split_wanted) cands.push_back({seq_c, true, vb_c});
      cands.push_back({seq_c, false, vb_c});
    }
  }
  P.waves = INT_MAX;
  for (const Cand &c : cands) {
    std::vector<size_t> b1;
    double a1 = 0.0;
    const int w1 = waves_for(c.seq, c.split, c.vb, b1, a1);
    if (w1 < P.waves) {
      P.waves = w1;
      P.seq = c.seq;
      P.split = c.split;
      P.vb = c.vb;
      P.bytes.swap(b1);
      P.all = a1;
    }
  }
  if (P.waves == INT_MAX) {
    const Cand c = cands.back();   // the smallest layout
    for (int i = 0; i < n_items; ++i) {
      const size_t need = theta_item_bytes(models[i]->host, need_selinv, c.seq, c.split, c.vb,
                                           twisted(models[i]->host, twist_ok));
      if ((double)need > budget)
        return fail(INLA_ERR_BUDGET, "item " + std::to_string(i) + " needs " + std::to_string(need) +
                                         " bytes, above the HBM budget");
    }
    return fail(INLA_ERR_BUDGET, "no layout fits the HBM budget");
  }
  return INLA_OK;
}

// One admission wave of a batched evaluation: the descriptors of every item's
// matrices, workspaces and outputs, laid out in one block of device memory
// (the library arena, or a block of its own when the factors are kept for a
// gradient asked for later).  Each matrix is one chain of time blocks, or two
// (a forward and a backward chain meeting at a middle block) when it is
// eliminated from both ends; the per-step phases run over the chains (*h
// batches), the arrow block, log-determinant and combination over the whole
// matrices.
struct Wave {
  int start = 0, k = 0;
  bool grad = false, need_selinv = false, seq = false, split = false, vb = false;
  bool twist_ok = false;   // matrices of four or more time blocks are eliminated from both ends
  bool io = false;       // theta and outputs in buffers of the wave (graph capture, kept factors)
  bool two_combines = false;   // also an f-only combination (gradient asked for later)
  bool want_var = false;
  std::vector<ThetaItemBufs> tb;
  std::vector<double *> Dbase;
  Batch F, Sv, Si, Fc, Sic;            // whole matrices
  Batch Fh, Svh, Sih, Fch, Sich;       // their chains
  Twist twf, twfc, twsi, twsic;        // matrices eliminated from both ends, per batch
  ItemDev *fdev = nullptr, *sdev = nullptr, *vdev = nullptr;
  ItemDev *fhdev = nullptr, *shdev = nullptr, *vhdev = nullptr;
  TwistPair *tpf = nullptr, *tpsi = nullptr;
  double **xs = nullptr, **tmps = nullptr, **xsh = nullptr, **tmpsh = nullptr, *logdet = nullptr;
  int *info = nullptr;
  TermItem *tdev = nullptr;
  CombineItem *cdev = nullptr;     // f, and the gradient when grad
  CombineItem *cdev_f = nullptr;   // f only (two_combines)
  EvalGraph G;                     // theta and outputs when io
  long long ntot = 0;              // length of the wave's mu / var outputs
};

// Workspace of a backward chain (its factor storage is the matrix's own).
void layout_back_ws(Layout &L, ItemDev &it, bool split, bool selinv) {
  const size_t bb = (size_t)it.b * it.b;
  L.add(&it.W1, bb);
  L.add(&it.W2, bb);
  L.add(&it.W3, std::max<size_t>((size_t)it.a * it.b, 1));
  L.add(&it.Mp, 2 * (size_t)kTile * kTile);
  if (split) L.add(&it.P, (size_t)kSplitK * bb);
  if (selinv) {
    L.add(&it.SD, 2 * bb);
    L.add(&it.SR, std::max<size_t>(2 * (size_t)it.a * it.b, 1));
  }
}

// Adds the wave's device buffers to L (the pointers are set once L is placed).
void wave_layout(Wave &W, const inla_model *const *models, bool mu_in_caller, Layout &L) {
  const int k = W.k;
  W.tb.assign(k, ThetaItemBufs());
  W.Dbase.assign(2 * k, nullptr);
  W.ntot = 0;
  for (int q = 0; q < k; ++q) W.ntot += models[W.start + q]->n;
  if (W.io) {
    L.add(&W.G.th, (size_t)4 * k);
    L.add(&W.G.f, (size_t)k);
    L.add(&W.G.g, (size_t)4 * k);
    L.add(&W.G.st, (size_t)k);
    L.add(&W.G.mu_buf, (size_t)W.ntot);
    if (W.want_var) L.add(&W.G.var_buf, (size_t)W.ntot);
  }
  for (int q = 0; q < k; ++q) {
    const ModelDev &h = models[W.start + q]->host;
    ThetaItemBufs &T = W.tb[q];
    T.tw = twisted(h, W.twist_ok);
    for (int w = 0; w < 2; ++w) {
      ItemDev &it = w ? T.C : T.P;
      ItemDev &bk = w ? T.Cb : T.Pb;
      std::memset(&it, 0, sizeof(it));
      std::memset(&bk, 0, sizeof(bk));
      it.b = h.b; it.nt = h.nt; it.a = h.a; it.nP = ntile(h.b);
      it.ntf = h.nt; it.nrun = h.nt; it.own_arrow = 1;
      it.sbw = band_aware() ? h.sbw : h.b;
      it.which = w;
      it.model = models[W.start + q]->dev;
      bk.b = h.b; bk.a = h.a; bk.nP = it.nP;
      if (w == 1 && W.seq) {
        // Q_c reuses the storage and workspaces of Q_prior (aliased in
        // wave_bind, once the memory is placed); only its trace partials are its own
        if (W.grad) L.add(&it.trpart, ((size_t)h.nt + 1) * kTraceBlocks * 4);
        continue;
      }
      L.add(&W.Dbase[2 * q + w], bta_doubles(h.b, h.nt, h.a));
      layout_factor_ws(L, it);
      if (W.split) L.add(&it.P, (size_t)kSplitK * h.b * h.b);
      if (W.need_selinv) {
        layout_selinv_ws(L, it);
        if (W.vb) {
          if (h.nt > 1) L.add(&it.V, (size_t)(h.nt - 1) * h.b * h.b);
          if (h.a > 0) L.add(&it.U, (size_t)h.nt * h.a * h.b);
          L.add(&it.G, (size_t)h.nt * h.b * h.b);
        }
        if (W.grad) L.add(&it.trpart, ((size_t)h.nt + 1) * kTraceBlocks * 4);
      }
      if (T.tw) {
        layout_back_ws(L, bk, W.split, W.need_selinv);
        if (h.a > 0) L.add(w ? &T.TBc : &T.TBp, (size_t)h.a * h.a);
      }
    }
    if (!mu_in_caller && !W.io) L.add(&T.x, (size_t)h.n);
    L.add(&T.tmp, (size_t)std::max(h.b, std::max(h.a, 1)));
    if (T.tw) L.add(&T.tmpb, (size_t)std::max(h.b, std::max(h.a, 1)));
    L.add(&T.term, (size_t)kTermBlocks * 4);
  }
  L.add(&W.fdev, 2 * k);
  L.add(&W.sdev, k);
  L.add(&W.vdev, 2 * k);
  L.add(&W.fhdev, 4 * k);
  L.add(&W.shdev, 2 * k);
  L.add(&W.vhdev, 4 * k);
  L.add(&W.tpf, 2 * k);
  L.add(&W.tpsi, 2 * k);
  L.add(&W.xs, k);
  L.add(&W.tmps, k);
  L.add(&W.xsh, 2 * k);
  L.add(&W.tmpsh, 2 * k);
  L.add(&W.logdet, 2 * k);
  L.add(&W.info, 2 * k);
  L.add(&W.tdev, k);
  L.add(&W.cdev, k);
  if (W.two_combines) L.add(&W.cdev_f, k);
}

// The forward chain (time blocks 0..m, m = ceil(nt/2)) of a whole matrix and
// its backward chain (blocks nt-1 down to m+1, whose last block is the
// middle one), completing bk, whose workspace is already placed; TB: its
// arrow accumulator.  The backward chain's last step updates the middle
// block in an earlier lockstep step than the forward chain's (nt-m-2 < m-1),
// so the two never touch it in one launch.
void make_chains(const ItemDev &full, ItemDev &fw, ItemDev &bk, double *TB, TwistPair &tp) {
  const int nt = full.nt, m = (nt + 1) / 2;
  const long long bb = (long long)full.b * full.b, ab = (long long)full.a * full.b;
  fw = full;
  fw.nt = m + 1; fw.nrun = m + 1; fw.own_arrow = 0;
  ItemDev w = bk;   // its workspace pointers
  bk = full;
  bk.W1 = w.W1; bk.W2 = w.W2; bk.W3 = w.W3; bk.Mp = w.Mp; bk.P = w.P;
  bk.SD = w.SD; bk.SR = w.SR;
  bk.SS = full.SS ? bk.W1 : nullptr;
  bk.nt = nt - m; bk.nrun = nt - m - 1; bk.ntf = nt; bk.trev = 1; bk.own_arrow = 0;
  bk.T = TB;
  bk.ldpart = full.ldpart + (long long)(m + 1) * full.nP;
  bk.trpart = full.trpart ? full.trpart + (long long)(m + 1) * kTraceBlocks * 4 : nullptr;
  bk.V = full.V ? full.V + (long long)m * bb : nullptr;
  bk.U = full.U ? full.U + (long long)(m + 1) * ab : nullptr;
  bk.G = full.G ? full.G + (long long)(m + 1) * bb : nullptr;
  std::memset(&tp, 0, sizeof(tp));
  tp.T = full.T; tp.TB = TB;
  if (full.SD) {
    tp.SDf = sig_D(fw, m); tp.SDb = sig_D(bk, bk.nt - 1);
    tp.SRf = sig_R(fw, m); tp.SRb = sig_R(bk, bk.nt - 1);
  }
  tp.a = full.a; tp.b = full.b; tp.m = m;
}

// Finishes the descriptors once the wave's memory is placed and uploads them.
// Without io the wave reads theta from theta_w and writes f, grad, status, mu
// and var straight to the caller's buffers (already offset to the wave).
// sigma (n = k, or null): caller storage that receives Sigma of Q_c.
inla_status wave_bind(Wave &W, const inla_model *const *models, const double *theta_w,
                      double *f_w, double *g_w, int *st_w, double *mu_w, double *var_w,
                      const inla_bta *sigma, hipStream_t s) {
  const int k = W.k;
  if (W.seq) {
    for (int q = 0; q < k; ++q) {
      ThetaItemBufs &T = W.tb[q];
      const ItemDev &pv = T.P;
      ItemDev &cv = T.C;
      cv.W1 = pv.W1; cv.W2 = pv.W2; cv.W3 = pv.W3; cv.Mp = pv.Mp; cv.P = pv.P;
      cv.ldpart = pv.ldpart; cv.info = pv.info;
      cv.SD = pv.SD; cv.SR = pv.SR; cv.ST = pv.ST; cv.V = pv.V; cv.U = pv.U; cv.G = pv.G;
      W.Dbase[2 * q + 1] = W.Dbase[2 * q];
      const ItemDev &pb = T.Pb;
      ItemDev &cb = T.Cb;
      cb.W1 = pb.W1; cb.W2 = pb.W2; cb.W3 = pb.W3; cb.Mp = pb.Mp; cb.P = pb.P;
      cb.SD = pb.SD; cb.SR = pb.SR;
      T.TBc = T.TBp;
    }
  }
  const double *th = W.io ? W.G.th : theta_w;
  double *fo = W.io ? W.G.f : f_w;
  double *go = W.io ? W.G.g : g_w;
  int *so = W.io ? W.G.st : st_w;
  double *muo = W.io ? W.G.mu_buf : mu_w;
  double *vo = W.io ? W.G.var_buf : var_w;
  W.F = Batch(); W.Sv = Batch(); W.Si = Batch(); W.Fc = Batch(); W.Sic = Batch();
  W.Fh = Batch(); W.Svh = Batch(); W.Sih = Batch(); W.Fch = Batch(); W.Sich = Batch();
  W.twf = Twist(); W.twfc = Twist(); W.twsi = Twist(); W.twsic = Twist();
  std::vector<double *> hx(k), ht(k), hxh, hth;
  std::vector<TermItem> thv(k);
  std::vector<CombineItem> ch(k), chf(k);
  auto add_twist = [](Twist &tw, const TwistPair &tp) {
    tw.host.push_back(tp);
    tw.max_a = std::max(tw.max_a, tp.a);
    tw.max_b = std::max(tw.max_b, tp.b);
  };
  long long off = 0;
  for (int q = 0; q < k; ++q) {
    const int i = W.start + q;
    const ModelDev &h = models[i]->host;
    ThetaItemBufs &T = W.tb[q];
    const size_t bb = (size_t)h.b * h.b;
    for (int w = 0; w < 2; ++w) {
      ItemDev &it = w ? T.C : T.P;
      double *base = W.Dbase[2 * q + w];
      it.D = base;
      it.S = h.nt > 1 ? base + (size_t)h.nt * bb : nullptr;
      it.R = h.a > 0 ? base + (size_t)(2 * h.nt - 1) * bb : nullptr;
      it.T = h.a > 0 ? it.R + (size_t)h.nt * h.a * h.b : nullptr;
      it.theta = th + 4 * q;
      if (W.need_selinv) it.SS = it.W1;
      if (w == 1 && vo) it.diag = vo + off;
      if (w == 1 && sigma) {
        // Sigma of Q_c into the caller's storage, every step's blocks kept
        const inla_bta &sg = sigma[q];
        it.SD = sg.D; it.sd_stride = (long long)bb;
        it.SS = sg.S; it.ss_stride = (long long)bb;
        it.SR = sg.R; it.sr_stride = (long long)h.a * h.b;
        it.ST = sg.T;
      }
    }
    if (muo) T.x = muo + off;
    hx[q] = T.x;
    ht[q] = T.tmp;
    // the chains of each matrix
    ItemDev pf = T.P, pb, cf = T.C, cb;
    TwistPair tpp, tpc;
    if (T.tw) {
      pb = T.Pb;
      cb = T.Cb;
      make_chains(T.P, pf, pb, T.TBp, tpp);
      make_chains(T.C, cf, cb, T.TBc, tpc);
    }
    auto chains = [&](Batch &B, const ItemDev &f, const ItemDev &bk) {
      B.host.push_back(f);
      if (T.tw) B.host.push_back(bk);
    };
    if (W.seq) {
      W.F.host.push_back(T.P);
      W.Fc.host.push_back(T.C);
      chains(W.Fh, pf, pb);
      chains(W.Fch, cf, cb);
      if (T.tw) {
        add_twist(W.twf, tpp);
        add_twist(W.twfc, tpc);
      }
      if (W.grad) {
        W.Si.host.push_back(T.P);
        chains(W.Sih, pf, pb);
        if (T.tw) add_twist(W.twsi, tpp);
      }
      if (W.need_selinv) {
        W.Sic.host.push_back(T.C);
        chains(W.Sich, cf, cb);
        if (T.tw) add_twist(W.twsic, tpc);
      }
    } else {
      W.F.host.push_back(T.P);
      W.F.host.push_back(T.C);
      chains(W.Fh, pf, pb);
      chains(W.Fh, cf, cb);
      if (T.tw) {
        add_twist(W.twf, tpp);
        add_twist(W.twf, tpc);
      }
      if (W.grad) {
        W.Si.host.push_back(T.P);
        chains(W.Sih, pf, pb);
        if (T.tw) add_twist(W.twsi, tpp);
      }
      if (W.need_selinv) {
        W.Si.host.push_back(T.C);
        chains(W.Sih, cf, cb);
        if (T.tw) add_twist(W.twsi, tpc);
      }
    }
    W.Sv.host.push_back(T.C);
    chains(W.Svh, cf, cb);
    hxh.push_back(T.x);
    hth.push_back(T.tmp);
    if (T.tw) {
      hxh.push_back(T.x);
      hth.push_back(T.tmpb);
    }
    thv[q] = TermItem{models[i]->dev, th + 4 * q, T.x, T.term};
    CombineItem c;
    std::memset(&c, 0, sizeof(c));
    c.model = models[i]->dev;
    c.theta = th + 4 * q;
    c.term_part = T.term;
    c.mu = T.x;
    c.logdet = W.logdet + 2 * q;
    c.info = W.info + 2 * q;
    c.f = fo + q;
    c.status = so ? so + q : nullptr;
    chf[q] = c;
    c.trp = W.grad ? T.P.trpart : nullptr;
    c.trc = W.grad ? T.C.trpart : nullptr;
    c.grad = (W.grad && go) ? go + 4 * q : nullptr;
    ch[q] = c;
    off += h.n;
  }
  // every descriptor must point into placed memory before anything is launched
  for (int q = 0; q < k; ++q) {
    const ThetaItemBufs &T = W.tb[q];
    for (const ItemDev *it : {&T.P, &T.C}) {
      const bool ok = it->D && it->W1 && it->W2 && it->W3 && it->Mp && it->ldpart && it->info &&
                      (!W.need_selinv || (it->SD && (it->a == 0 || (it->SR && it->ST)))) &&
                      (!W.grad || it->trpart) && T.x && T.tmp && T.term;
      if (!ok) return fail(INLA_ERR_STATE, "internal: workspace of item " +
                                               std::to_string(W.start + q) + " not placed");
    }
    if (T.tw) {
      const bool ok = T.Pb.W1 && T.Pb.W2 && T.Pb.W3 && T.Pb.Mp && T.tmpb &&
                      (!W.need_selinv || T.Pb.SD) && (T.P.a == 0 || T.TBp);
      if (!ok) return fail(INLA_ERR_STATE, "internal: chain workspace of item " +
                                               std::to_string(W.start + q) + " not placed");
    }
  }
  // descriptor arrays: the sequential layout splits them in halves
  W.F.dev = W.fdev; W.Sv.dev = W.sdev; W.Si.dev = W.vdev;
  W.Fc.dev = W.fdev + k; W.Sic.dev = W.vdev + k;
  W.Fh.dev = W.fhdev; W.Svh.dev = W.shdev; W.Sih.dev = W.vhdev;
  W.Fch.dev = W.fhdev + 2 * k; W.Sich.dev = W.vhdev + 2 * k;
  W.twf.dev = W.tpf; W.twsi.dev = W.tpsi;
  W.twfc.dev = W.tpf + k; W.twsic.dev = W.tpsi + k;
  for (Batch *B : {&W.F, &W.Sv, &W.Si, &W.Fh, &W.Svh, &W.Sih}) B->finalize();
  if (W.seq)
    for (Batch *B : {&W.Fc, &W.Sic, &W.Fch, &W.Sich}) B->finalize();
  for (Batch *B : {&W.Si, &W.Sic, &W.Sih, &W.Sich}) B->vb = W.vb;
  // the chains of a matrix use the tile choice of the whole matrices
  for (Batch *B : {&W.Fh, &W.Svh, &W.Sih, &W.Fch, &W.Sich}) B->big = W.F.big;
  ST_TRY(upload(W.fdev, W.F.host, s));
  ST_TRY(upload(W.fhdev, W.Fh.host, s));
  if (W.seq) {
    ST_TRY(upload(W.Fc.dev, W.Fc.host, s));
    ST_TRY(upload(W.Fch.dev, W.Fch.host, s));
  }
  ST_TRY(upload(W.sdev, W.Sv.host, s));
  ST_TRY(upload(W.shdev, W.Svh.host, s));
  if (W.need_selinv && !W.Si.host.empty()) {
    ST_TRY(upload(W.vdev, W.Si.host, s));
    ST_TRY(upload(W.vhdev, W.Sih.host, s));
  }
  if (W.seq && W.need_selinv) {
    ST_TRY(upload(W.Sic.dev, W.Sic.host, s));
    ST_TRY(upload(W.Sich.dev, W.Sich.host, s));
  }
  ST_TRY(upload(W.tpf, W.twf.host, s));
  ST_TRY(upload(W.tpsi, W.twsi.host, s));
  if (W.seq) {
    ST_TRY(upload(W.twfc.dev, W.twfc.host, s));
    ST_TRY(upload(W.twsic.dev, W.twsic.host, s));
  }
  ST_TRY(upload(W.xs, hx, s));
  ST_TRY(upload(W.tmps, ht, s));
  ST_TRY(upload(W.xsh, hxh, s));
  ST_TRY(upload(W.tmpsh, hth, s));
  ST_TRY(upload(W.tdev, thv, s));
  ST_TRY(upload(W.cdev, ch, s));
  if (W.two_combines) ST_TRY(upload(W.cdev_f, chf, s));
  return INLA_OK;
}

inla_status wave_assemble(Wave &W, const inla_model *const *models, int w, hipStream_t ls) {
  for (int q = 0; q < W.k; ++q) {
    const int i = W.start + q;
    const ModelDev &h = models[i]->host;
    ItemDev &it = w ? W.tb[q].C : W.tb[q].P;
    {
      ProfScope ps(PS_ASSEMBLE, 0.0, ls);
      HIP_TRY(launch_assemble(models[i]->dev, h.b, h.nt, h.a, it.theta, w, it.D, it.S, it.R, it.T,
                              w ? W.tb[q].x : nullptr, ls));
    }
    HIP_TRY(launch_fill_int(it.info, 1, kInfoNone, ls));
  }
  return INLA_OK;
}

// The wave's launches.  defer_grad: the two-matrix layout runs everything but
// the selected inversions, and combines f only (wave_gradient runs the rest).
inla_status wave_forward(Wave &W, const inla_model *const *models, bool defer_grad, hipStream_t ls) {
  const int k = W.k;
  if (!W.seq) {
    // assemble Q_prior, Q_c and b = tau_y A^T y (into x, solved in place)
    ST_TRY(wave_assemble(W, models, 0, ls));
    ST_TRY(wave_assemble(W, models, 1, ls));
    ST_TRY(run_factor(W.Fh, W.F, W.twf, ls));
    HIP_TRY(launch_logdet_finish(W.fdev, 2 * k, W.logdet, W.info, ls));
    if (W.need_selinv && !defer_grad) {
      // the mode solve (and its terms) beside the selected inversion: both
      // only read the factor, and they write disjoint buffers
      HIP_TRY(hipEventRecord(g_solve_fork, ls));
      HIP_TRY(hipStreamWaitEvent(g_solve, g_solve_fork, 0));
      ST_TRY(run_solve(W.Svh, W.Sv, W.xsh, W.tmpsh, W.xs, W.tmps, g_solve));
      HIP_TRY(launch_terms(W.tdev, k, g_solve));
      HIP_TRY(hipEventRecord(g_solve_join, g_solve));
      ST_TRY(run_selinv(W.Sih, W.Si, W.twsi, true, ls));
      HIP_TRY(hipStreamWaitEvent(ls, g_solve_join, 0));
    } else {
      ST_TRY(run_solve(W.Svh, W.Sv, W.xsh, W.tmpsh, W.xs, W.tmps, ls));
      HIP_TRY(launch_terms(W.tdev, k, ls));
    }
  } else {
    if (defer_grad) return fail(INLA_ERR_STATE, "internal: shared storage cannot keep both factors");
    // Q_prior first (factor, log-determinant, gradient traces), then Q_c
    // in the same storage
    ST_TRY(wave_assemble(W, models, 0, ls));
    ST_TRY(run_factor(W.Fh, W.F, W.twf, ls));
    HIP_TRY(launch_logdet_finish(W.fdev, k, W.logdet, W.info, ls, 2));
    if (W.grad) ST_TRY(run_selinv(W.Sih, W.Si, W.twsi, true, ls));
    ST_TRY(wave_assemble(W, models, 1, ls));
    ST_TRY(run_factor(W.Fch, W.Fc, W.twfc, ls));
    HIP_TRY(launch_logdet_finish(W.Fc.dev, k, W.logdet + 1, W.info + 1, ls, 2));
    ST_TRY(run_solve(W.Svh, W.Sv, W.xsh, W.tmpsh, W.xs, W.tmps, ls));
    HIP_TRY(launch_terms(W.tdev, k, ls));
    if (W.need_selinv) ST_TRY(run_selinv(W.Sich, W.Sic, W.twsic, true, ls));
  }
  HIP_TRY(launch_combine(defer_grad ? W.cdev_f : W.cdev, k, ls));
  return INLA_OK;
}

// The deferred half of a two-matrix wave: both selected inversions with their
// traces, then f and the gradient combined (the same launches, in the same
// order per matrix, as the one-pass evaluation).
inla_status wave_gradient(Wave &W, hipStream_t ls) {
  ST_TRY(run_selinv(W.Sih, W.Si, W.twsi, true, ls));
  HIP_TRY(launch_combine(W.cdev, W.k, ls));
  return INLA_OK;
}

// One batched evaluation with a fixed tile choice.  `seq_mode`: 2 never,
// 1 always, 0 when the two-matrix layout needs more admission waves than the
// one-matrix layout.  sigma (n_items, or null): Sigma of each item's Q_c into
// caller storage (then nothing is captured in a graph).
inla_status eval_run(const inla_model *const *models, int32_t n_items, const double *theta_dev,
                     double *f_dev, double *grad_dev, double *mu_out, double *var_out,
                     int32_t *status_dev, const inla_bta *sigma, double budget, int seq_mode,
                     bool allow_graph, hipStream_t s) {
  const bool grad = grad_dev != nullptr;
  const bool need_selinv = grad || var_out != nullptr || sigma != nullptr;
  const bool twist_ok = twist_env() && sigma == nullptr;
  EvalPlan plan;
  ST_TRY(plan_eval(models, n_items, grad, need_selinv, budget, seq_mode, twist_ok, plan));
  // per-item output offsets into the concatenated mu / var buffers
  std::vector<long long> voff(n_items + 1, 0);
  for (int i = 0; i < n_items; ++i) voff[i + 1] = voff[i] + models[i]->n;
  const long long ntot = voff[n_items];
  const int tile = tile_request(), variant = big_variant(), small = small_variant(),
            step = step_fused_override();

  // replay a captured graph when the call matches it and nothing else has
  // laid out the workspace since
  // (events recorded during capture cannot be timed, so profiling runs eagerly)
  const bool graphable = allow_graph && graphs_enabled() && !g_prof.on && plan.all <= budget &&
                         sigma == nullptr;
  GraphKey key;
  for (int i = 0; i < n_items; ++i) {
    const ModelDev &h = models[i]->host;
    key.model_ids.push_back(models[i]->id);
    for (int64_t v : {(int64_t)h.b, (int64_t)h.nt, (int64_t)h.a, (int64_t)models[i]->n})
      key.shapes.push_back(v);
  }
  key.grad = grad; key.var = var_out != nullptr; key.mu = mu_out != nullptr; key.prof = g_prof.on;
  key.seq = plan.seq; key.split = plan.split; key.vb = plan.vb; key.twist = twist_ok;
  key.band = band_aware();
  key.tile = tile; key.variant = variant; key.small = small; key.step = step;
  key.gen = g_arena.gen; key.base = g_arena.base; key.ntot = ntot;
  if (graphable && g_graph.valid && same_signature(g_graph.key, key)) {
    if (g_arena.last && g_arena.last_stream != s) HIP_TRY(hipStreamWaitEvent(s, g_arena.last, 0));
    HIP_TRY(hipMemcpyAsync(g_graph.th, theta_dev, (size_t)n_items * 32, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipGraphLaunch(g_graph.exec, s));
    ST_TRY(copy_outputs(g_graph, n_items, ntot, f_dev, grad_dev, mu_out, var_out, status_dev, s));
    return arena_done(s);
  }
  if (graphable) drop_graph();

  int start = 0;
  while (start < n_items) {
    int end = start;
    double acc = 0.0;
    while (end < n_items && acc + (double)plan.bytes[end] <= budget) acc += (double)plan.bytes[end++];
    Wave W;
    W.start = start;
    W.k = end - start;
    W.grad = grad; W.need_selinv = need_selinv;
    W.seq = plan.seq; W.split = plan.split; W.vb = plan.vb;
    W.twist_ok = twist_ok;
    W.io = graphable;
    W.want_var = var_out != nullptr;
    Layout L;
    wave_layout(W, models, mu_out != nullptr, L);
    ST_TRY(arena_bind(L, s));
    ST_TRY(wave_bind(W, models, theta_dev + 4 * start, f_dev + start,
                     grad ? grad_dev + 4 * start : nullptr, status_dev ? status_dev + start : nullptr,
                     mu_out ? mu_out + voff[start] : nullptr, var_out ? var_out + voff[start] : nullptr,
                     sigma ? sigma + start : nullptr, s));
    if (graphable)
      HIP_TRY(hipMemcpyAsync(W.G.th, theta_dev, (size_t)W.k * 32, hipMemcpyDeviceToDevice, s));
    hipStream_t ls = s;
    if (graphable) {
      ls = g_cap;
      HIP_TRY(hipStreamBeginCapture(ls, hipStreamCaptureModeThreadLocal));
    }
    if (g_prof.on) ++g_prof.calls;
    inla_status st = wave_forward(W, models, false, ls);
    if (graphable) {
      hipGraph_t graph = nullptr;
      hipError_t e = hipStreamEndCapture(ls, &graph);
      if (st != INLA_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
      }
      if (e != hipSuccess) return fail(INLA_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
      hipGraphExec_t exec = nullptr;
      e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) return fail(INLA_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(e));
      EvalGraph G = W.G;
      G.valid = true;
      G.exec = exec;
      G.key = key;
      // the arena was laid out afresh for this call: the key takes its new state
      G.key.gen = g_arena.gen;
      G.key.base = g_arena.base;
      g_graph = G;
      HIP_TRY(hipGraphLaunch(g_graph.exec, s));
      ST_TRY(copy_outputs(g_graph, n_items, ntot, f_dev, grad_dev, mu_out, var_out, status_dev, s));
    } else if (st != INLA_OK) {
      return st;
    }
    start = end;
  }
  return arena_done(s);
}

// ---------------------------------------------------------------------------
// autotuner: per call signature, the tile layout of the b x b products is
// timed once for each candidate and the fastest is kept in memory and in a
// small JSON file (one entry per line) that later processes read back
// ---------------------------------------------------------------------------
struct TileChoice {
  int tile = 0;      // 64 or 128 (0: built-in rule)
  int variant = kDefaultBigVariant;   // layout of the 128-wide kernel
  int small = kDefaultSmallVariant;   // form of the 64-wide product phases
  int step = -1;     // Cholesky step: 1 fused, 0 batched, -1 the tile-count rule
  double ms = 0.0;
};
std::unordered_map<std::string, TileChoice> g_tune;
std::string g_tune_loaded;

std::string tune_key(const inla_model *const *models, int n, bool grad, bool var) {
  // the multiset of item shapes, order-free
  std::vector<std::string> shapes;
  for (int i = 0; i < n; ++i) {
    const ModelDev &h = models[i]->host;
    shapes.push_back(std::to_string(h.b) + "x" + std::to_string(h.nt) + "x" + std::to_string(h.a));
  }
  std::sort(shapes.begin(), shapes.end());
  std::string all;
  for (auto &x : shapes) all += x + ",";
  unsigned long long hsh = 1469598103934665603ULL;   // FNV-1a
  for (unsigned char c : all) hsh = (hsh ^ c) * 1099511628211ULL;
  char buf[96];
  snprintf(buf, sizeof(buf), "%s:n%d:%s:%016llx", grad ? "grad" : (var ? "var" : "f"), n,
           shapes.back().c_str(), hsh);
  return buf;
}

void tune_load(const std::string &path) {
  if (g_tune_loaded == path) return;
  g_tune_loaded = path;
  FILE *fp = fopen(path.c_str(), "r");
  if (!fp) return;
  char line[512];
  while (fgets(line, sizeof(line), fp)) {
    char key[256];
    TileChoice c;
    const int got = sscanf(line,
                           " \"%255[^\"]\": {\"tile\": %d, \"variant\": %d, \"small\": %d, "
                           "\"step\": %d, \"ms\": %lf",
                           key, &c.tile, &c.variant, &c.small, &c.step, &c.ms);
    if (got == 6 && (c.tile == 64 || c.tile == 128) && c.variant >= 0 && c.variant < kBigVariants &&
        c.small >= 0 && c.small < kSmallVariants && c.step >= -1 && c.step <= 1)
      g_tune[key] = c;
  }
  fclose(fp);
}

void tune_save(const std::string &path) {
  const std::string tmp = path + ".tmp";
  FILE *fp = fopen(tmp.c_str(), "w");
  if (!fp) return;
  std::vector<std::string> keys;
  for (auto &kv : g_tune) keys.push_back(kv.first);
  std::sort(keys.begin(), keys.end());
  fprintf(fp, "{\n");
  for (size_t i = 0; i < keys.size(); ++i) {
    const TileChoice &c = g_tune[keys[i]];
    fprintf(fp, "  \"%s\": {\"tile\": %d, \"variant\": %d, \"small\": %d, \"step\": %d, \"ms\": %.4f}%s\n",
            keys[i].c_str(), c.tile, c.variant, c.small, c.step, c.ms, i + 1 < keys.size() ? "," : "");
  }
  fprintf(fp, "}\n");
  fclose(fp);
  (void)rename(tmp.c_str(), path.c_str());
}

inla_status check_opts(const inla_opts *opts) {
  if (!opts) return INLA_OK;
  if (opts->keep_sigma != 0 && opts->keep_sigma != 1) return fail(INLA_ERR_ARG, "keep_sigma must be 0 or 1");
  if (opts->tile != 0 && opts->tile != 64 && opts->tile != 128)
    return fail(INLA_ERR_ARG, "tile must be 0, 64 or 128");
  if (opts->recompute < 0 || opts->recompute > 2)
    return fail(INLA_ERR_ARG, "recompute must be 0, 1 or 2");
  return INLA_OK;
}

// The HBM budget of a call: the caller's, else free memory plus the arena
// minus a 4 GiB reserve.
inla_status call_budget(const inla_opts *opts, double *budget) {
  *budget = opts ? opts->hbm_budget_bytes : 0.0;
  if (!(*budget > 0.0)) {
    size_t fr = 0, tot = 0;
    HIP_TRY(hipMemGetInfo(&fr, &tot));
    *budget = (double)fr + (double)g_arena.cap - 4.0 * (1ULL << 30);
  }
  return INLA_OK;
}

inla_status eval_impl(const inla_model *const *models, int32_t n_items, const double *theta_dev,
                      double *f_dev, double *grad_dev, double *mu_out, double *var_out,
                      int32_t *status_dev, const inla_opts *opts, hipStream_t s) {
  if (!models || n_items < 1 || !theta_dev || !f_dev)
    return fail(INLA_ERR_ARG, "need models, n_items >= 1, theta and f");
  for (int i = 0; i < n_items; ++i)
    if (!models[i]) return fail(INLA_ERR_ARG, "NULL model in batch");
  ST_TRY(check_opts(opts));
  const inla_bta *sigma = nullptr;
  if (opts && opts->keep_sigma == 1) {
    if (!opts->sigma_out) return fail(INLA_ERR_ARG, "keep_sigma = 1 needs sigma_out");
    for (int i = 0; i < n_items; ++i) {
      ST_TRY(check_bta(&opts->sigma_out[i], "sigma_out"));
      const ModelDev &h = models[i]->host;
      if (opts->sigma_out[i].b != h.b || opts->sigma_out[i].nt != h.nt || opts->sigma_out[i].a != h.a)
        return fail(INLA_ERR_ARG, "sigma_out[" + std::to_string(i) + "] shape does not match the model");
    }
    sigma = opts->sigma_out;
  }
  ST_TRY(ensure_streams());
  double budget = 0.0;
  ST_TRY(call_budget(opts, &budget));
  const int seq_mode = opts ? opts->recompute : 0;
  auto run = [&](const TileChoice &c, bool allow_graph) -> inla_status {
    g_tile_pref = c.tile;
    set_big_variant(c.variant);
    set_small_variant(c.small);
    g_step_pref = c.step;
    const inla_status st = eval_run(models, n_items, theta_dev, f_dev, grad_dev, mu_out, var_out,
                                    status_dev, sigma, budget, seq_mode, allow_graph, s);
    g_tile_pref = 0;
    set_big_variant(kDefaultBigVariant);
    set_small_variant(kDefaultSmallVariant);
    g_step_pref = -1;
    return st;
  };
  TileChoice choice;
  if (opts && opts->tile != 0) {
    choice.tile = opts->tile;
  } else if (opts && opts->autotune_cache && opts->autotune_cache[0]) {
    const std::string path = opts->autotune_cache;
    tune_load(path);
    const std::string key = tune_key(models, n_items, grad_dev != nullptr, var_out != nullptr);
    auto itc = g_tune.find(key);
    if (itc != g_tune.end()) {
      choice = itc->second;
    } else {
      // time every candidate eagerly (one untimed run, one timed) on the
      // caller's stream; every run computes the same outputs
      TileChoice cands[kSmallVariants + kBigVariants];
      for (int v = 0; v < kSmallVariants; ++v) {
        cands[v].tile = 64;
        cands[v].small = v;
      }
      for (int v = 0; v < kBigVariants; ++v) {
        cands[kSmallVariants + v].tile = 128;
        cands[kSmallVariants + v].variant = v;
      }
      hipEvent_t e0, e1;
      HIP_TRY(hipEventCreate(&e0));
      HIP_TRY(hipEventCreate(&e1));
      bool have = false;
      auto trial = [&](TileChoice c) -> inla_status {
        inla_status st = run(c, false);
        if (st == INLA_OK) {
          HIP_TRY(hipEventRecord(e0, s));
          st = run(c, false);
          HIP_TRY(hipEventRecord(e1, s));
        }
        if (st != INLA_OK) return st;
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        c.ms = ms;
        if (!have || c.ms < choice.ms) choice = c;
        have = true;
        return INLA_OK;
      };
      // the product layouts under the tile-count rule for the step form, then
      // both step forms with the best layout
      inla_status st = INLA_OK;
      for (const TileChoice &c0 : cands)
        if (st == INLA_OK) st = trial(c0);
      for (int form = 0; form <= 1 && st == INLA_OK; ++form) {
        TileChoice c = choice;
        c.step = form;
        st = trial(c);
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      if (st != INLA_OK) return st;
      g_tune[key] = choice;
      tune_save(path);
    }
  }
  return run(choice, true);
}


// Tile choice of a call: the caller's tile, else the autotuner's stored entry
// for the call's signature, else the built-in rule (nothing is timed here).
TileChoice stored_choice(const inla_model *const *models, int n, const inla_opts *opts, bool grad,
                         bool var) {
  TileChoice c;
  if (opts && opts->tile != 0) {
    c.tile = opts->tile;
  } else if (opts && opts->autotune_cache && opts->autotune_cache[0]) {
    tune_load(opts->autotune_cache);
    auto it = g_tune.find(tune_key(models, n, grad, var));
    if (it != g_tune.end()) c = it->second;
  }
  return c;
}

struct ChoiceScope {
  explicit ChoiceScope(const TileChoice &c) {
    g_tile_pref = c.tile;
    set_big_variant(c.variant);
    set_small_variant(c.small);
  }
  ~ChoiceScope() {
    g_tile_pref = 0;
    set_big_variant(kDefaultBigVariant);
    set_small_variant(kDefaultSmallVariant);
  }
};

}  // namespace

// f now, its gradient later: the factors of a batch kept between the two.
struct inla_eval_state {
  std::vector<const inla_model *> models;
  int n = 0;
  bool kept = false;           // factors kept (else the gradient recomputes everything)
  void *mem = nullptr;         // device block: the kept wave, or the theta copy
  double *theta = nullptr;     // the theta batch (device copy)
  Wave W;
  TileChoice choice;
  inla_opts opts{};
  std::string cache;
  int device = 0;
  hipEvent_t done = nullptr;   // completion of the last call on the state
};

namespace {

inla_status state_record(inla_eval_state *st, hipStream_t s) {
  if (!st->done) HIP_TRY(hipEventCreateWithFlags(&st->done, hipEventDisableTiming));
  HIP_TRY(hipEventRecord(st->done, s));
  return INLA_OK;
}

inla_status eval_f_keep_impl(const inla_model *const *models, int32_t n_items,
                             const double *theta_dev, double *f_dev, double *mu_out,
                             int32_t *status_dev, const inla_opts *opts, hipStream_t s,
                             inla_eval_state **out) {
  if (!out) return fail(INLA_ERR_ARG, "state_out must be non-NULL");
  *out = nullptr;
  if (!models || n_items < 1 || !theta_dev || !f_dev)
    return fail(INLA_ERR_ARG, "need models, n_items >= 1, theta and f");
  for (int i = 0; i < n_items; ++i)
    if (!models[i]) return fail(INLA_ERR_ARG, "NULL model in batch");
  ST_TRY(check_opts(opts));
  if (opts && opts->keep_sigma) return fail(INLA_ERR_ARG, "keep_sigma is for inla_eval_f_grad");
  ST_TRY(ensure_streams());
  double budget = 0.0;
  ST_TRY(call_budget(opts, &budget));
  auto *st = new inla_eval_state();
  st->models.assign(models, models + n_items);
  st->n = n_items;
  if (opts) {
    st->opts = *opts;
    if (opts->autotune_cache) {
      st->cache = opts->autotune_cache;
      st->opts.autotune_cache = st->cache.c_str();
    }
    st->opts.sigma_out = nullptr;
  }
  HIP_TRY(hipGetDevice(&st->device));
  st->choice = stored_choice(models, n_items, opts, true, false);
  inla_status rc = INLA_OK;
  {
    ChoiceScope cs(st->choice);
    // the gradient's layout, both matrices in storage of their own, one wave
    EvalPlan plan;
    if ((!opts || opts->recompute != 1) &&
        plan_eval(models, n_items, true, true, budget, 2, twist_env(), plan) == INLA_OK &&
        plan.waves == 1) {
      Wave &W = st->W;
      W.start = 0;
      W.k = n_items;
      W.grad = true; W.need_selinv = true;
      W.seq = false; W.split = plan.split; W.vb = plan.vb;
      W.twist_ok = plan.twist_ok;
      W.io = true;
      W.want_var = true;
      W.two_combines = true;
      Layout L;
      wave_layout(W, models, false, L);
      void *p = nullptr;
      if (hipMalloc(&p, align_up(L.total)) == hipSuccess) {
        st->mem = p;
        size_t off = 0;
        for (auto &r : L.reqs) {
          *r.slot = static_cast<char *>(p) + off;
          off += align_up(std::max<size_t>(r.bytes, 1));
        }
        st->kept = true;
      } else {
        (void)hipGetLastError();
      }
    }
    g_last_error.clear();
    if (st->kept) {
      Wave &W = st->W;
      st->theta = W.G.th;
      rc = wave_bind(W, models, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, s);
      if (rc == INLA_OK) {
        const auto D2D = hipMemcpyDeviceToDevice;
        hipError_t e = hipMemcpyAsync(W.G.th, theta_dev, (size_t)n_items * 32, D2D, s);
        if (e != hipSuccess) rc = fail(INLA_ERR_HIP, std::string("theta copy: ") + hipGetErrorString(e));
        if (rc == INLA_OK) {
          if (g_prof.on) ++g_prof.calls;
          rc = wave_forward(W, models, true, s);
        }
        if (rc == INLA_OK) {
          e = hipMemcpyAsync(f_dev, W.G.f, (size_t)n_items * 8, D2D, s);
          if (!e && status_dev) e = hipMemcpyAsync(status_dev, W.G.st, (size_t)n_items * 4, D2D, s);
          if (!e && mu_out) e = hipMemcpyAsync(mu_out, W.G.mu_buf, (size_t)W.ntot * 8, D2D, s);
          if (e != hipSuccess) rc = fail(INLA_ERR_HIP, std::string("output copy: ") + hipGetErrorString(e));
        }
      }
    }
  }
  if (rc == INLA_OK && !st->kept) {
    // not kept: f as usual now, everything again for the gradient
    void *p = nullptr;
    if (hipMalloc(&p, (size_t)n_items * 32) != hipSuccess) {
      (void)hipGetLastError();
      delete st;
      return fail(INLA_ERR_NOMEM, "theta copy allocation failed");
    }
    st->mem = p;
    st->theta = static_cast<double *>(p);
    hipError_t e = hipMemcpyAsync(st->theta, theta_dev, (size_t)n_items * 32,
                                  hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) rc = fail(INLA_ERR_HIP, std::string("theta copy: ") + hipGetErrorString(e));
    if (rc == INLA_OK)
      rc = eval_impl(models, n_items, theta_dev, f_dev, nullptr, mu_out, nullptr, status_dev, opts, s);
  }
  if (rc == INLA_OK) rc = state_record(st, s);
  if (rc != INLA_OK) {
    (void)hipDeviceSynchronize();
    if (st->mem) (void)hipFree(st->mem);
    delete st;
    return rc;
  }
  *out = st;
  return INLA_OK;
}

inla_status eval_grad_kept_impl(inla_eval_state *st, double *f_dev, double *grad_dev,
                                double *var_out, int32_t *status_dev, hipStream_t s) {
  if (!st) return fail(INLA_ERR_ARG, "state is NULL");
  if (!f_dev || !grad_dev) return fail(INLA_ERR_ARG, "f_dev and grad_dev must be non-NULL");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != st->device) return fail(INLA_ERR_STATE, "state belongs to another device");
  if (st->done) HIP_TRY(hipStreamWaitEvent(s, st->done, 0));
  if (!st->kept) {
    // the factors were not kept: the whole evaluation again
    ST_TRY(eval_impl(st->models.data(), st->n, st->theta, f_dev, grad_dev, nullptr, var_out,
                     status_dev, &st->opts, s));
    return state_record(st, s);
  }
  ST_TRY(ensure_streams());
  Wave &W = st->W;
  {
    ChoiceScope cs(st->choice);
    if (g_prof.on) ++g_prof.calls;
    ST_TRY(wave_gradient(W, s));
  }
  const auto D2D = hipMemcpyDeviceToDevice;
  const int n = st->n;
  HIP_TRY(hipMemcpyAsync(f_dev, W.G.f, (size_t)n * 8, D2D, s));
  HIP_TRY(hipMemcpyAsync(grad_dev, W.G.g, (size_t)n * 32, D2D, s));
  if (status_dev) HIP_TRY(hipMemcpyAsync(status_dev, W.G.st, (size_t)n * 4, D2D, s));
  if (var_out) HIP_TRY(hipMemcpyAsync(var_out, W.G.var_buf, (size_t)W.ntot * 8, D2D, s));
  return state_record(st, s);
}

}  // namespace

extern "C" {

inla_status inla_eval_f(const inla_model *const *models, int32_t n_items, const double *theta_dev,
                        double *f_dev, double *mu_or_null, double *var_or_null, int32_t *status_dev,
                        const inla_opts *opts, void *hip_stream) {
  g_last_error.clear();
  std::lock_guard<std::mutex> lk(g_mutex);
  return eval_impl(models, n_items, theta_dev, f_dev, nullptr, mu_or_null, var_or_null, status_dev,
                   opts, static_cast<hipStream_t>(hip_stream));
}

inla_status inla_eval_f_grad(const inla_model *const *models, int32_t n_items,
                             const double *theta_dev, double *f_dev, double *grad_dev,
                             double *mu_or_null, double *var_or_null, int32_t *status_dev,
                             const inla_opts *opts, void *hip_stream) {
  g_last_error.clear();
  if (!grad_dev) return fail(INLA_ERR_ARG, "grad_dev must be non-NULL");
  std::lock_guard<std::mutex> lk(g_mutex);
  return eval_impl(models, n_items, theta_dev, f_dev, grad_dev, mu_or_null, var_or_null,
                   status_dev, opts, static_cast<hipStream_t>(hip_stream));
}

inla_status inla_eval_f_keep(const inla_model *const *models, int32_t n_items,
                             const double *theta_dev, double *f_dev, double *mu_or_null,
                             int32_t *status_dev, const inla_opts *opts, void *hip_stream,
                             inla_eval_state **state_out) {
  g_last_error.clear();
  std::lock_guard<std::mutex> lk(g_mutex);
  return eval_f_keep_impl(models, n_items, theta_dev, f_dev, mu_or_null, status_dev, opts,
                          static_cast<hipStream_t>(hip_stream), state_out);
}

inla_status inla_eval_grad_kept(inla_eval_state *state, double *f_dev, double *grad_dev,
                                double *var_or_null, int32_t *status_dev, void *hip_stream) {
  g_last_error.clear();
  std::lock_guard<std::mutex> lk(g_mutex);
  return eval_grad_kept_impl(state, f_dev, grad_dev, var_or_null, status_dev,
                             static_cast<hipStream_t>(hip_stream));
}

int32_t inla_eval_state_kept(const inla_eval_state *state) { return state && state->kept ? 1 : 0; }

void inla_eval_state_destroy(inla_eval_state *state) {
  if (!state) return;
  if (state->done) {
    (void)hipEventSynchronize(state->done);
    (void)hipEventDestroy(state->done);
  }
  if (state->mem) (void)hipFree(state->mem);
  delete state;
}

inla_status inla_profile_begin(void) {
  std::lock_guard<std::mutex> lk(g_mutex);
  drop_graph();   // a captured graph may hold events of the pool
  g_prof.recs.clear();
  g_prof.used = 0;
  g_prof.calls = 0;
  g_prof.on = true;
  return INLA_OK;
}

inla_status inla_profile_end(double *out, int32_t nslots) {
  std::lock_guard<std::mutex> lk(g_mutex);
  g_prof.on = false;
  const int nall = PS_COUNT + 1 + PK_COUNT;
  std::vector<double> acc(3 * nall, 0.0);
  int bad = 0;
  for (auto &r : g_prof.recs) {
    float ms = 0.f;
    if (hipEventSynchronize(r.e1) != hipSuccess || hipEventElapsedTime(&ms, r.e0, r.e1) != hipSuccess) {
      (void)hipGetLastError();
      ++bad;
      continue;
    }
    for (int slot : {r.slot, PS_COUNT + 1 + r.kind}) {
      acc[3 * slot + 0] += 1.0;
      acc[3 * slot + 1] += ms;
      acc[3 * slot + 2] += r.flops;
    }
  }
  // slot PS_COUNT: evaluations represented, unreadable records
  acc[3 * PS_COUNT + 0] = g_prof.calls;
  acc[3 * PS_COUNT + 1] = bad;
  g_prof.recs.clear();
  g_prof.used = 0;
  drop_graph();
  if (out)
    for (int k = 0; k < std::min<int>(nslots, nall) * 3; ++k) out[k] = acc[k];
  return INLA_OK;
}

int32_t inla_profile_slots(void) { return PS_COUNT + 1 + PK_COUNT; }

void inla_release_workspace(void) {
  std::lock_guard<std::mutex> lk(g_mutex);
  drop_graph();
  if (g_arena.base) {
    (void)hipDeviceSynchronize();
    (void)hipFree(g_arena.base);
    g_arena.base = nullptr;
    g_arena.cap = 0;
  }
}

}  // extern "C"
