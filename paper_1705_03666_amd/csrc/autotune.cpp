// Default launch schedules.  The search over schedules lives in the Python
// autotuner (paper_1705_03666_amd/autotune.py), which times candidates through
// the option overrides and caches the winner per device and problem shape;
// whatever it passes in pdd_options takes precedence here.
#include "pdd_tuning.hpp"

#include <algorithm>

namespace pdd {

Tuning choose_tuning(int dim, bool fp32, bool adjoint, const pdd_options& o, int n_cus, int64_t total_paths) {
  (void)dim;
  (void)adjoint;
  Tuning t;
  // measured on MI355X for the 3-D C5 walk (forward and adjoint alike)
  t.chunk_paths = 16384;
  t.blocks_per_cu = fp32 ? 8 : 4;
  t.refill_groups = 3;
  if (o.blocks_per_cu > 0) t.blocks_per_cu = o.blocks_per_cu;
  if (o.refill_groups > 0) t.refill_groups = o.refill_groups;
  if (o.chunk_paths > 0) {
    t.chunk_paths = o.chunk_paths;
  } else {
    // a call too small for the default items: halve the item size (down to
    // 1024 paths) until every resident wavefront gets about four items
    const int64_t waves = (int64_t)t.blocks_per_cu * std::max(1, n_cus) * 4;
    while (t.chunk_paths > 1024 && total_paths / t.chunk_paths < 4 * waves) t.chunk_paths /= 2;
  }
  t.chunk_paths = std::max(1, t.chunk_paths);
  return t;
}

Tuning choose_branch_tuning(int dim, bool fp32, const pdd_options& o, int n_cus, int64_t total_trees) {
  (void)dim;
  Tuning t;
  // measured on MI355X for C4 / C7 (k_branch) and C6 (k_branch_bvp), 1024
  // points x 1e5 trees: four blocks per CU (the FP32 kernels are built for
  // four waves per SIMD: at most 128 VGPRs and 37 KB of LDS per block) and
  // items of 16384 trees, so a wavefront merges its Welford triple into an
  // item slot rarely; 2 blocks and 2048-tree items took 2.0x (C4) and 1.2x
  // (C6) as long
  t.chunk_paths = 16384;
  t.blocks_per_cu = fp32 ? 4 : 2;
  t.refill_groups = 1;
  if (o.blocks_per_cu > 0) t.blocks_per_cu = o.blocks_per_cu;
  if (o.chunk_paths > 0) {
    t.chunk_paths = o.chunk_paths;
  } else {
    // smaller calls: halve the item size (down to 1024 trees) until every
    // resident wavefront gets at least one item
    const int64_t waves = (int64_t)t.blocks_per_cu * std::max(1, n_cus) * 4;
    while (t.chunk_paths > 1024 && total_trees / t.chunk_paths < waves) t.chunk_paths /= 2;
  }
  t.chunk_paths = std::max(1, t.chunk_paths);
  return t;
}

}  // namespace pdd
