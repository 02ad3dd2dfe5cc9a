// Device buffers of one host-side call (host-only helper of the drivers
// around the evaluation path), freed on every return path.
#ifndef INLA_CALL_BUFFERS_H
#define INLA_CALL_BUFFERS_H

#include <hip/hip_runtime.h>

#include <cstddef>
#include <vector>

namespace inla {

struct CallBuffers {
  std::vector<void *> p;
  CallBuffers() = default;
  CallBuffers(const CallBuffers &) = delete;
  CallBuffers &operator=(const CallBuffers &) = delete;
  ~CallBuffers() {
    for (void *q : p)
      if (q) (void)hipFree(q);
  }
  template <class T>
  bool get(T **out, size_t count) {
    void *q = nullptr;
    if (hipMalloc(&q, (count > 0 ? count : 1) * sizeof(T)) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    p.push_back(q);
    *out = static_cast<T *>(q);
    return true;
  }
};

}  // namespace inla

#endif  // INLA_CALL_BUFFERS_H
