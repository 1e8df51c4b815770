// Launch schedule of the persistent kernels: paths per work item, persistent
// grid size, and how many step groups run between lane refills.  Values come
// from the caller's options when set, else from the tuned table
// (autotune.cpp), else from built-in defaults.
#pragma once
#include <stdint.h>

#include "pdd.h"

namespace pdd {

struct Tuning {
  int chunk_paths;
  int blocks_per_cu;
  int refill_groups;
};

// total_paths: paths of the whole call (sizes the default work item so that
// small calls still give every resident wavefront several items).
Tuning choose_tuning(int dim, bool fp32, bool adjoint, const pdd_options& o, int n_cus, int64_t total_paths);
Tuning choose_branch_tuning(int dim, bool fp32, const pdd_options& o, int n_cus, int64_t total_trees);

}  // namespace pdd
