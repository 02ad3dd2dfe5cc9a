// Host check of the task order of a Cholesky step launch (csrc/inla_internal.h):
// for every tile count up to 40, both step forms (the batched left-looking one
// and the fused right-looking one) and every tile column, the long-first
// numbering (step_split / step_task_local) is a bijection onto the decoder's
// task numbers 0 .. phase_tasks - 1, and nothing runs past the chain's steps.
#include "inla_internal.h"
#include <cstdio>
#include <vector>
using namespace inla;
int main() {
  int bad = 0, cases = 0;
  for (int nP = 1; nP <= 40; ++nP)
    for (int ph : {PH_STEP, PH_STEPF})
      for (int p = 0; p <= nP; ++p) {
        ItemDev it{};
        it.nP = nP; it.nt = 3; it.nrun = 3; it.b = nP * 64; it.a = 2;
        const int tot = phase_tasks(it, ph, 1, p);
        StepSplit z = step_split(nP, ph, 1, p, 3);
        if (z.nlong() + z.nshort() != tot) { printf("count mismatch nP=%d ph=%d p=%d: %d+%d vs %d\n", nP, ph, p, z.nlong(), z.nshort(), tot); ++bad; }
        std::vector<int> seen(tot, 0);
        for (int c = 0; c < z.nlong(); ++c) { int q = step_task_local(z, true, c); if (q < 0 || q >= tot) { ++bad; printf("range\n"); } else seen[q]++; }
        for (int c = 0; c < z.nshort(); ++c) { int q = step_task_local(z, false, c); if (q < 0 || q >= tot) { ++bad; printf("range\n"); } else seen[q]++; }
        for (int q = 0; q < tot; ++q) if (seen[q] != 1) { ++bad; printf("q %d seen %d (nP=%d ph=%d p=%d)\n", q, seen[q], nP, ph, p); }
        ++cases;
        // past nrun: nothing
        StepSplit z2 = step_split(nP, ph, 3, p, 3);
        if (z2.nlong() + z2.nshort() != 0) ++bad;
      }
  printf("%d cases, %d problems\n", cases, bad);
  if (!bad) printf("step split checks passed\n");
  return bad != 0;
}
