// Adjoint instantiations of the walk kernel, FP64 stepping.
#include <hip/hip_runtime.h>

#include "walk_kernels.hpp"

namespace pdd {

template <typename R, int DIM, int DFC, int LAYOUT, int NT, bool ADJ>
static hipError_t launch_walk_t(const WalkLaunch& L, hipStream_t st) {
  hipLaunchKernelGGL((k_walk<R, DIM, DFC, LAYOUT, NT, ADJ>), dim3(L.grid), dim3(kBlock), 0, st, *L.P, L.items,
                     L.n_items, L.qhead, L.istat, L.igrad, L.grad_stride, L.dump_phi, L.dump_steps, L.dump_off,
                     L.refill_groups);
  return hipGetLastError();
}

template <typename R, int LAYOUT, int NT, bool ADJ>
static hipError_t launch_walk_dim(const WalkLaunch& L, hipStream_t st) {
  const bool poly = L.dfc >= 0;
  switch (L.P->dim) {
    case 1: return poly ? launch_walk_t<R, 1, 3, LAYOUT, NT, ADJ>(L, st) : launch_walk_t<R, 1, -1, LAYOUT, NT, ADJ>(L, st);
    case 2: return poly ? launch_walk_t<R, 2, 3, LAYOUT, NT, ADJ>(L, st) : launch_walk_t<R, 2, -1, LAYOUT, NT, ADJ>(L, st);
    default: return poly ? launch_walk_t<R, 3, 3, LAYOUT, NT, ADJ>(L, st) : launch_walk_t<R, 3, -1, LAYOUT, NT, ADJ>(L, st);
  }
}

hipError_t launch_walk_adj_f64(const WalkLaunch& L, hipStream_t st) {
  if (L.P->layout == RNG_QUAD24)
    return L.nt > 0 ? launch_walk_dim<double, RNG_QUAD24, kAdjTerms, true>(L, st)
                    : launch_walk_dim<double, RNG_QUAD24, 0, true>(L, st);
  return L.nt > 0 ? launch_walk_dim<double, RNG_PAIR52, kAdjTerms, true>(L, st)
                  : launch_walk_dim<double, RNG_PAIR52, 0, true>(L, st);
}

}  // namespace pdd
