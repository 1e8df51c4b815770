// Forward (value-only) instantiations of the walk kernels and the plain FP64 baseline.
#include <hip/hip_runtime.h>

#include "walk_kernels.hpp"

namespace pdd {

template <typename R, int LAYOUT>
static hipError_t launch_wos_dim(const WalkLaunch& L, hipStream_t st) {
  switch (L.P->dim) {
    case 1: return launch_walk_t<R, 1, -1, LAYOUT, false, false, true>(L, st);
    case 2: return launch_walk_t<R, 2, -1, LAYOUT, false, false, true>(L, st);
    default: return launch_walk_t<R, 3, -1, LAYOUT, false, false, true>(L, st);
  }
}

// Walk on spheres (Laplace's equation; b = c = f = 0).
hipError_t launch_walk_wos(const WalkLaunch& L, hipStream_t st) {
  if (L.fp32) return launch_wos_dim<float, RNG_QUAD24>(L, st);
  if (L.P->layout == RNG_QUAD24) return launch_wos_dim<double, RNG_QUAD24>(L, st);
  return launch_wos_dim<double, RNG_PAIR52>(L, st);
}

hipError_t launch_walk_fwd(const WalkLaunch& L, hipStream_t st) {
  if (L.fp32) return launch_walk_terms<float, RNG_QUAD24, false>(L, st);
  if (L.P->layout == RNG_QUAD24) return launch_walk_terms<double, RNG_QUAD24, false>(L, st);
  return launch_walk_terms<double, RNG_PAIR52, false>(L, st);
}

template <int DIM, int DFC, int LAYOUT>
static hipError_t launch_plain_t(const PlainLaunch& L, hipStream_t st) {
  hipLaunchKernelGGL((k_walk_plain<DIM, DFC, LAYOUT>), dim3(L.grid), dim3(kBlock), 0, st, *L.P, L.node, L.n_paths,
                     L.bstat, L.dump_phi, L.dump_steps, L.dump_base);
  return hipGetLastError();
}

template <int LAYOUT>
static hipError_t launch_plain_l(const PlainLaunch& L, hipStream_t st) {
  const bool poly = L.dfc >= 0;
  switch (L.P->dim) {
    case 1: return poly ? launch_plain_t<1, 3, LAYOUT>(L, st) : launch_plain_t<1, -1, LAYOUT>(L, st);
    case 2: return poly ? launch_plain_t<2, 3, LAYOUT>(L, st) : launch_plain_t<2, -1, LAYOUT>(L, st);
    default: return poly ? launch_plain_t<3, 3, LAYOUT>(L, st) : launch_plain_t<3, -1, LAYOUT>(L, st);
  }
}

hipError_t launch_plain(const PlainLaunch& L, hipStream_t st) {
  return L.P->layout == RNG_QUAD24 ? launch_plain_l<RNG_QUAD24>(L, st) : launch_plain_l<RNG_PAIR52>(L, st);
}

}  // namespace pdd
