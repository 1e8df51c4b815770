// Adjoint instantiations of the walk kernel, FP64 stepping.
#include <hip/hip_runtime.h>

#include "walk_kernels.hpp"

namespace pdd {

hipError_t launch_walk_adj_f64(const WalkLaunch& L, hipStream_t st) {
  if (L.P->layout == RNG_QUAD24) return launch_walk_terms<double, RNG_QUAD24, true>(L, st);
  return launch_walk_terms<double, RNG_PAIR52, true>(L, st);
}

template <int DIM, int DFC, int LAYOUT, int NT>
static hipError_t launch_plain_adj_t(const PlainLaunch& L, hipStream_t st) {
  hipLaunchKernelGGL((k_walk_plain_adj<DIM, DFC, LAYOUT, NT>), dim3(L.grid), dim3(kBlock), 0, st, *L.P, L.node,
                     L.n_paths, L.bstat, L.brow, L.grad_stride);
  return hipGetLastError();
}

template <int LAYOUT, int NT>
static hipError_t launch_plain_adj_l(const PlainLaunch& L, hipStream_t st) {
  const bool poly = L.dfc >= 0;
  switch (L.P->dim) {
    case 1: return poly ? launch_plain_adj_t<1, 3, LAYOUT, NT>(L, st) : launch_plain_adj_t<1, -1, LAYOUT, NT>(L, st);
    case 2: return poly ? launch_plain_adj_t<2, 3, LAYOUT, NT>(L, st) : launch_plain_adj_t<2, -1, LAYOUT, NT>(L, st);
    default: return poly ? launch_plain_adj_t<3, 3, LAYOUT, NT>(L, st) : launch_plain_adj_t<3, -1, LAYOUT, NT>(L, st);
  }
}

// FP64 plain adjoint: one node per launch (the single-node baseline).
hipError_t launch_plain_adj(const PlainLaunch& L, hipStream_t st) {
  if (L.P->layout == RNG_QUAD24)
    return L.nt > 0 ? launch_plain_adj_l<RNG_QUAD24, kAdjTerms>(L, st) : launch_plain_adj_l<RNG_QUAD24, 0>(L, st);
  return L.nt > 0 ? launch_plain_adj_l<RNG_PAIR52, kAdjTerms>(L, st) : launch_plain_adj_l<RNG_PAIR52, 0>(L, st);
}

}  // namespace pdd
