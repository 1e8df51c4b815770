// Adjoint instantiations of the walk kernel, FP32 stepping.
#include <hip/hip_runtime.h>

#include "walk_kernels.hpp"

namespace pdd {

hipError_t launch_walk_adj_f32(const WalkLaunch& L, hipStream_t st) {
  return launch_walk_terms<float, RNG_QUAD24, true>(L, st);
}

}  // namespace pdd
