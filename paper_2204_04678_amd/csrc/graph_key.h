// The call signature a captured evaluation graph is valid for (host-only C++,
// no HIP: unit-tested on the CPU by compiling it with g++).
//
// A captured graph bakes in the device addresses of the models' data, of the
// library workspace and of every per-item descriptor.  It may be replayed only
// for a call that would have recorded the same launches on the same memory:
// the same models (by identity, never by host address: a new model can be
// allocated at the address of a destroyed one), the same shapes, the same
// outputs asked for, the same layout choices and the same workspace layout.
#ifndef INLA_GRAPH_KEY_H
#define INLA_GRAPH_KEY_H

#include <cstdint>
#include <vector>

namespace inla {

struct GraphKey {
  std::vector<uint64_t> model_ids;   // per item: the model's creation id (never reused)
  std::vector<int64_t> shapes;       // per item: b, nt, a, n
  bool grad = false, var = false, mu = false, prof = false;
  bool seq = false, split = false, vb = false, twist = false, band = false;
  int tile = 0, variant = 0, small = 0, step = -1;
  uint64_t gen = 0;                  // workspace layout generation
  const void *base = nullptr;        // workspace base address
  int64_t ntot = 0;                  // total length of the mu / var outputs
};

inline bool same_signature(const GraphKey &x, const GraphKey &y) {
  return x.model_ids == y.model_ids && x.shapes == y.shapes && x.grad == y.grad &&
         x.var == y.var && x.mu == y.mu && x.prof == y.prof && x.seq == y.seq &&
         x.split == y.split && x.vb == y.vb && x.twist == y.twist && x.band == y.band && x.tile == y.tile &&
         x.variant == y.variant &&
         x.small == y.small && x.step == y.step && x.gen == y.gen && x.base == y.base &&
         x.ntot == y.ntot;
}

// True when a graph with key x reads the data of the model with this id.
inline bool key_uses_model(const GraphKey &x, uint64_t id) {
  for (uint64_t m : x.model_ids)
    if (m == id) return true;
  return false;
}

}  // namespace inla

#endif  // INLA_GRAPH_KEY_H
