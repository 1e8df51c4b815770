// Adjoint instantiations of the walk kernel, FP64 stepping.
#include <hip/hip_runtime.h>

#include "walk_kernels.hpp"

namespace pdd {

hipError_t launch_walk_adj_f64(const WalkLaunch& L, hipStream_t st) {
  if (L.P->layout == RNG_QUAD24) return launch_walk_terms<double, RNG_QUAD24, true>(L, st);
  return launch_walk_terms<double, RNG_PAIR52, true>(L, st);
}

}  // namespace pdd
