// FP32 p-multigrid state (device buffers owned by the context).
#pragma once
#include <hip/hip_runtime.h>

namespace pfmf {

struct MGState {
  int n_levels = 0;
};

inline void mg_free(MGState& mg) { mg.n_levels = 0; }

}  // namespace pfmf
