// Launchers of the branching kernels (Sec. 3.1-3.2) with psi and g read from
// the staged term table; a problem-specialised instantiation compiled at run
// time is launched through the module API instead (BranchLaunch::spec).
#include <hip/hip_runtime.h>

#include "branch_kernels.hpp"
#include "pdd_kernels.hpp"

namespace pdd {

template <typename R, int LAYOUT>
static hipError_t launch_branch_bvp_t(const BranchBvpLaunch& L, hipStream_t st) {
  switch (L.P->dim) {
    case 1:
      hipLaunchKernelGGL((k_branch_bvp<R, 1, LAYOUT>), dim3(L.grid), dim3(kBlock), 0, st, *L.P, *L.B, L.items,
                         L.n_items, L.qhead, L.istat, L.dump_val, L.dump_segs, L.trees, (StackEntry<R>*)L.stack,
                         L.stack_entries);
      break;
    case 2:
      hipLaunchKernelGGL((k_branch_bvp<R, 2, LAYOUT>), dim3(L.grid), dim3(kBlock), 0, st, *L.P, *L.B, L.items,
                         L.n_items, L.qhead, L.istat, L.dump_val, L.dump_segs, L.trees, (StackEntry<R>*)L.stack,
                         L.stack_entries);
      break;
    default:
      hipLaunchKernelGGL((k_branch_bvp<R, 3, LAYOUT>), dim3(L.grid), dim3(kBlock), 0, st, *L.P, *L.B, L.items,
                         L.n_items, L.qhead, L.istat, L.dump_val, L.dump_segs, L.trees, (StackEntry<R>*)L.stack,
                         L.stack_entries);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_branch_bvp(const BranchBvpLaunch& L, hipStream_t st) {
  if (L.spec != nullptr) {
    // same argument list as k_branch_bvp; the parameter blocks are passed by value
    const WorkItem* items = L.items;
    int n_items = L.n_items;
    uint32_t* qhead = L.qhead;
    ItemStat* istat = L.istat;
    double* dump_val = L.dump_val;
    int64_t* dump_segs = L.dump_segs;
    int64_t trees = L.trees, stack_entries = L.stack_entries;
    void* stack = L.stack;
    void* args[] = {(void*)L.P, (void*)L.B, &items, &n_items, &qhead, &istat, &dump_val, &dump_segs,
                    &trees, &stack, &stack_entries};
    return hipModuleLaunchKernel(L.spec, (unsigned)L.grid, 1, 1, kBlock, 1, 1, 0, st, args, nullptr);
  }
  if (L.fp32) return launch_branch_bvp_t<float, RNG_QUAD24>(L, st);
  if (L.layout == RNG_QUAD24) return launch_branch_bvp_t<double, RNG_QUAD24>(L, st);
  return launch_branch_bvp_t<double, RNG_PAIR52>(L, st);
}

template <typename R, int LAYOUT>
static hipError_t launch_branch_t(const BranchLaunch& L, hipStream_t st) {
  switch (L.P->dim) {
    case 1:
      hipLaunchKernelGGL((k_branch<R, 1, LAYOUT>), dim3(L.grid), dim3(kBlock), 0, st, *L.P, L.items, L.n_items,
                         L.qhead, L.istat, L.dump_val, L.dump_segs, L.trees, (StackEntry<R>*)L.stack,
                         L.stack_entries);
      break;
    case 2:
      hipLaunchKernelGGL((k_branch<R, 2, LAYOUT>), dim3(L.grid), dim3(kBlock), 0, st, *L.P, L.items, L.n_items,
                         L.qhead, L.istat, L.dump_val, L.dump_segs, L.trees, (StackEntry<R>*)L.stack,
                         L.stack_entries);
      break;
    default:
      hipLaunchKernelGGL((k_branch<R, 3, LAYOUT>), dim3(L.grid), dim3(kBlock), 0, st, *L.P, L.items, L.n_items,
                         L.qhead, L.istat, L.dump_val, L.dump_segs, L.trees, (StackEntry<R>*)L.stack,
                         L.stack_entries);
      break;
  }
  return hipGetLastError();
}

size_t branch_stack_entry_bytes(bool fp32) { return fp32 ? sizeof(StackEntry<float>) : sizeof(StackEntry<double>); }
int branch_lds_depth(bool fp32) { return fp32 ? lds_depth<float>() : lds_depth<double>(); }

hipError_t launch_branch(const BranchLaunch& L, hipStream_t st) {
  if (L.spec != nullptr) {
    // same argument list as k_branch; the parameter block is passed by value
    const WorkItem* items = L.items;
    int n_items = L.n_items;
    uint32_t* qhead = L.qhead;
    ItemStat* istat = L.istat;
    double* dump_val = L.dump_val;
    int64_t* dump_segs = L.dump_segs;
    int64_t trees = L.trees, stack_entries = L.stack_entries;
    void* stack = L.stack;
    void* args[] = {(void*)L.P, &items, &n_items, &qhead, &istat, &dump_val, &dump_segs, &trees, &stack,
                    &stack_entries};
    return hipModuleLaunchKernel(L.spec, (unsigned)L.grid, 1, 1, kBlock, 1, 1, 0, st, args, nullptr);
  }
  if (L.fp32) return launch_branch_t<float, RNG_QUAD24>(L, st);
  if (L.layout == RNG_QUAD24) return launch_branch_t<double, RNG_QUAD24>(L, st);
  return launch_branch_t<double, RNG_PAIR52>(L, st);
}

}  // namespace pdd
