// Launch descriptors and launcher entry points of the HIP kernels (host side).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pdd_internal.hpp"

namespace pdd {

// Device mirror of pdd_node_stat (40 bytes).
struct pdd_node_stat_dev {
  double mean, m2;
  int64_t n, steps, censored;
};

struct WalkLaunch {
  const LinearParams* P;
  int dfc;                   // -1: no polynomial part in b, c, f; else 3
  bool terms;                // b, c, f (adjoint: or g) have generic terms; adjoint rows then carry
                             // kAdjTerms term columns per function
  bool fp32;
  bool adjoint;
  bool wos;                  // walk on spheres (b = c = f = 0; P->dt holds eps)
  hipFunction_t spec;        // problem-specialised k_walk (runtime-compiled), or null
  int grid;
  const WorkItem* items;
  int n_items;
  uint32_t* qhead;
  ItemStat* istat;
  double* igrad;
  int grad_stride;
  double* dump_phi;
  int64_t* dump_steps;
  const int64_t* dump_off;
  int refill_groups;
};

// Heterogeneous batch (walk_batch.hip): per-problem records, node -> problem.
struct WalkBatchLaunch {
  const LinearParams* probs;   // device [n_problems]
  const int32_t* node_prob;    // device [n_nodes]
  const double* nodes;         // device [n_nodes][3]
  const DevFactor* fac;
  const double* cd;
  const float* cf;
  uint32_t key0, key1;
  bool fp32;
  int layout;
  bool wos;
  int grid;
  const WorkItem* items;
  int n_items;
  uint32_t* qhead;
  ItemStat* istat;
  double* dump_phi;
  int64_t* dump_steps;
  const int64_t* dump_off;
  int refill_groups;
};

struct PlainLaunch {
  const LinearParams* P;
  int dfc;
  int grid;
  int node;
  uint32_t n_paths;
  ItemStat* bstat;
  double* dump_phi;
  int64_t* dump_steps;
  int64_t dump_base;
  // adjoint: one derivative row per block
  bool adjoint;
  int nt;                    // generic-term tangent slots (0 or kAdjTerms)
  double* brow;
  int grad_stride;
};

struct BranchLaunch {
  const BranchParams* P;
  bool fp32;
  int layout;
  int grid;
  const WorkItem* items;
  int n_items;
  uint32_t* qhead;
  ItemStat* istat;
  double* dump_val;
  int64_t* dump_segs;
  int64_t trees;
  void* stack;               // spill stack for deep trees
  int64_t stack_entries;     // entries per lane
  hipFunction_t spec;        // problem-specialised k_branch (same arguments), or null
};

// Branching with a Dirichlet boundary and output times; istat is
// [n_times][n_items].
struct BranchBvpLaunch {
  const BranchParams* P;
  const BranchBoundary* B;
  bool fp32;
  int layout;
  int grid;
  const WorkItem* items;
  int n_items;
  uint32_t* qhead;
  ItemStat* istat;
  double* dump_val;          // [points][trees][n_times]
  int64_t* dump_segs;        // [points][trees]
  int64_t trees;
  void* stack;
  int64_t stack_entries;
  hipFunction_t spec;        // problem-specialised k_branch_bvp (same arguments), or null
};

hipError_t launch_walk(const WalkLaunch& L, hipStream_t st);
hipError_t launch_walk_batch(const WalkBatchLaunch& L, hipStream_t st);
hipError_t launch_plain(const PlainLaunch& L, hipStream_t st);
hipError_t launch_plain_adj(const PlainLaunch& L, hipStream_t st);
hipError_t launch_branch(const BranchLaunch& L, hipStream_t st);
hipError_t launch_branch_bvp(const BranchBvpLaunch& L, hipStream_t st);
size_t branch_stack_entry_bytes(bool fp32);
// LDS stack entries per lane of k_branch and k_branch_bvp
int branch_lds_depth(bool fp32);
hipError_t launch_finalize_nodes(const ItemStat* istat, const int64_t* first, int64_t n_nodes, const CallPtrs* cp,
                                 int64_t out_off, unsigned long long* counters, hipStream_t st);
hipError_t launch_finalize_grad(const double* igrad, int stride, int n_cols, int n_items, const int32_t* slot_node,
                                const CallPtrs* cp, const double* inv_n, double* colsum, hipStream_t st);
hipError_t launch_node_jacobian(const double* igrad, int stride, const int64_t* first, int64_t n_nodes,
                                const double* inv_n, const int32_t* colmap, int n_cols, const CallPtrs* cp,
                                int64_t jac_ld, hipStream_t st);
hipError_t launch_scatter_add(const double* src, const int32_t* map, int count, const CallPtrs* cp, int which,
                              hipStream_t st);
// grad = J^T w, or with data != nullptr the misfit gradient (w_i = 2 (mean_i - data_i))
// and loss = sum_i (mean_i - data_i)^2
hipError_t launch_jacobian_apply(const double* jac, int64_t n_rows, int64_t ld, int64_t n_cols, const double* w,
                                 const void* stats, const double* data, double* grad, double* loss, hipStream_t st);
hipError_t launch_node_moments(const void* stats, int64_t n, double* var, double* se, hipStream_t st);
hipError_t launch_merge_estimates(void* acc, double* acc_jac, int64_t acc_ld, const void* add, const double* add_jac,
                                  int64_t add_ld, int64_t n_params, const int64_t* index, int64_t n_add,
                                  hipStream_t st);
hipError_t launch_stage(const StageJob* jobs, int n_jobs, const int32_t* perm, double* cd, float* cf,
                        hipStream_t st);
hipError_t launch_fill_u32(uint32_t* p, int n, uint32_t v, hipStream_t st);
hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t st);

}  // namespace pdd
