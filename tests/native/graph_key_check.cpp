// Host-only check of the captured-graph key (csrc/graph_key.h): a graph is
// replayed only for the same models by creation id, never for another model
// that happens to reuse a destroyed model's host address, and never for
// another output size.  Prints one line per failed check; exit status 0 when
// every check holds.
#include <cstdio>

#include "graph_key.h"

using inla::GraphKey;

static int failures = 0;
static void check(bool ok, const char *what) {
  if (!ok) {
    std::printf("FAILED: %s\n", what);
    ++failures;
  }
}

static GraphKey key_for(std::vector<uint64_t> ids, std::vector<int64_t> shapes, int64_t ntot) {
  GraphKey k;
  k.model_ids = ids;
  k.shapes = shapes;
  k.grad = true;
  k.mu = true;
  k.var = true;
  k.tile = 64;
  k.gen = 7;
  k.base = reinterpret_cast<const void *>(0x1000);
  k.ntot = ntot;
  return k;
}

int main() {
  // model A (id 1): b = 16, nt = 3, a = 2, n = 50
  const GraphKey a = key_for({1}, {16, 3, 2, 50}, 50);
  check(inla::same_signature(a, a), "a key matches itself");
  check(inla::same_signature(a, key_for({1}, {16, 3, 2, 50}, 50)), "equal keys match");
  // model B created after A was destroyed, with another id and shape
  const GraphKey b = key_for({2}, {25, 3, 0, 75}, 75);
  check(!inla::same_signature(a, b), "another model does not match");
  // the same shape under another id (a new model at a reused address) must not match
  check(!inla::same_signature(a, key_for({2}, {16, 3, 2, 50}, 50)),
        "same shape, other model id does not match");
  // same id with another output size (cannot happen for one model; still refused)
  check(!inla::same_signature(a, key_for({1}, {16, 3, 2, 50}, 51)), "other ntot does not match");
  // each flag and layout field takes part in the comparison
  GraphKey c = a;
  c.grad = false;
  check(!inla::same_signature(a, c), "grad flag");
  c = a; c.var = false;
  check(!inla::same_signature(a, c), "var flag");
  c = a; c.mu = false;
  check(!inla::same_signature(a, c), "mu flag");
  c = a; c.seq = true;
  check(!inla::same_signature(a, c), "storage mode");
  c = a; c.vb = true;
  check(!inla::same_signature(a, c), "selected-inversion form");
  c = a; c.twist = true;
  check(!inla::same_signature(a, c), "elimination order");
  c = a; c.band = true;
  check(!inla::same_signature(a, c), "band-aware products");
  c = a; c.tile = 128;
  check(!inla::same_signature(a, c), "tile");
  c = a; c.step = 1;
  check(!inla::same_signature(a, c), "step form");
  c = a; c.gen = 8;
  check(!inla::same_signature(a, c), "workspace generation");
  c = a; c.base = reinterpret_cast<const void *>(0x2000);
  check(!inla::same_signature(a, c), "workspace base");
  // batches: order matters (outputs are per item)
  const GraphKey ab = key_for({1, 2}, {16, 3, 2, 50, 25, 3, 0, 75}, 125);
  const GraphKey ba = key_for({2, 1}, {25, 3, 0, 75, 16, 3, 2, 50}, 125);
  check(!inla::same_signature(ab, ba), "item order");
  // which graphs a destroyed model invalidates
  check(inla::key_uses_model(ab, 1) && inla::key_uses_model(ab, 2), "batch uses both models");
  check(!inla::key_uses_model(a, 2), "single-model graph does not use model 2");
  check(!inla::key_uses_model(GraphKey(), 1), "empty key uses no model");
  if (failures == 0) std::printf("graph key checks passed\n");
  return failures == 0 ? 0 : 1;
}
