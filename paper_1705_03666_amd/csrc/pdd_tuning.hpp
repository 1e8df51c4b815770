// Launch schedule of the persistent kernels: paths (trees) per work item,
// persistent grid size, and how many step groups run between lane refills.
// Each knob comes from the caller's options when set, else from the device's
// tuned table (schedule.cpp), else from built-in defaults.
#pragma once
#include <stdint.h>

#include "pdd.h"

namespace pdd {

struct Tuning {
  int chunk_paths;
  int blocks_per_cu;
  int refill_groups;
};

// kernel: pdd_kernel; precision: PDD_FP64 or PDD_FP32_STEP; total_work: paths
// (trees) of the whole call, which sizes the default work item so that small
// calls still give every resident wavefront several items.
Tuning choose_schedule(int kernel, int dim, int precision, const pdd_options& o, int n_cus, int64_t total_work);

bool schedule_kind_valid(int kernel, int dim, int precision);
int set_schedule(int kernel, int dim, int precision, const pdd_launch_schedule* s);  // s == nullptr: remove; -1 if invalid
int get_schedule(int kernel, int dim, int precision, pdd_launch_schedule* out, int32_t* tuned);
int save_schedules(const char* path);   // nullptr: the default file; -1 on failure
int load_schedules(const char* path);   // entries read, -1 if the file cannot be read

}  // namespace pdd
