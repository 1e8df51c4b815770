// Reduction, staging and fill kernels shared by all entry points, and the
// dispatch of the walk launch to its instantiation unit.
#include <hip/hip_runtime.h>

#include "pdd_device.hpp"
#include "pdd_kernels.hpp"

namespace pdd {

// ---------------------------------------------------------------------------
// Merge item partials into per-node statistics in item-slot order (fixed).
__global__ void k_finalize_nodes(const ItemStat* __restrict__ istat, const int64_t* __restrict__ first,
                                 int64_t n_nodes, const CallPtrs* __restrict__ cp, int64_t out_off,
                                 unsigned long long* __restrict__ counters) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_nodes) return;
  pdd_node_stat_dev* __restrict__ out = (pdd_node_stat_dev*)cp->out + out_off;
  double n = 0.0, m = 0.0, q = 0.0;
  int64_t st = 0, ce = 0, rd = 0;
  for (int64_t s = first[i]; s < first[i + 1]; ++s) {
    const ItemStat v = istat[s];
    chan_merge(n, m, q, (double)v.n, v.mean, v.m2);
    st += v.steps;
    ce += v.censored;
    rd += v.redrawn;
  }
  pdd_node_stat_dev r;
  r.mean = m; r.m2 = q; r.n = (int64_t)n; r.steps = st; r.censored = ce;
  out[i] = r;
  if (counters != nullptr && (ce != 0 || rd != 0)) {
    if (ce) atomicAdd(&counters[0], (unsigned long long)ce);
    if (rd) atomicAdd(&counters[1], (unsigned long long)rd);
  }
}

// Adjoint reduction: grad[k] = sum over items s (in slot order) of
// (w[node_s] / N[node_s]) * row_s[k]; one block per column, fixed tree order.
__global__ void k_finalize_grad(const double* __restrict__ igrad, int stride, int n_items,
                                const int32_t* __restrict__ slot_node, const CallPtrs* __restrict__ cp,
                                const double* __restrict__ inv_n, double* __restrict__ colsum) {
  const int col = blockIdx.x;
  const double* __restrict__ w = cp->w;
  __shared__ double part[kBlock];
  double acc = 0.0;
  for (int s = threadIdx.x; s < n_items; s += blockDim.x) {
    const int nd = slot_node[s];
    acc += (w[nd] * inv_n[nd]) * igrad[(size_t)s * stride + col];
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) colsum[col] = part[0];
}

// Per-node Jacobian: jac[i][c] = (1/N_i) * sum over the items of node i (slot
// order) of row_s[colmap[c]].  One block per node.
__global__ void k_node_jacobian(const double* __restrict__ igrad, int stride, const int64_t* __restrict__ first,
                                const double* __restrict__ inv_n, const int32_t* __restrict__ colmap, int n_cols,
                                const CallPtrs* __restrict__ cp, int64_t jac_ld) {
  const int64_t i = blockIdx.x;
  double* __restrict__ jac = cp->jac;
  for (int c = threadIdx.x; c < n_cols; c += blockDim.x) {
    const int src = colmap[c];
    double acc = 0.0;
    for (int64_t s = first[i]; s < first[i + 1]; ++s) acc += igrad[(size_t)s * stride + src];
    jac[(size_t)i * jac_ld + c] = acc * inv_n[i];
  }
}

// dst[map[k]] += src[k] for the gradient columns of one coefficient array
// (dst = the caller's array number `which` of the call block).
__global__ void k_scatter_add(const double* __restrict__ src, const int32_t* __restrict__ map, int count,
                              const CallPtrs* __restrict__ cp, int which) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  double* __restrict__ dst = cp->grad[which];
  if (k < count) dst[map ? map[k] : k] += src[k];
}

// Copy the caller's coefficient arrays into the staged FP64/FP32 tables.
__global__ void k_stage(const StageJob* __restrict__ jobs, int n_jobs, const int32_t* __restrict__ perm,
                        double* __restrict__ cd, float* __restrict__ cf) {
  for (int j = 0; j < n_jobs; ++j) {
    const StageJob J = jobs[j];
    if (J.dst != nullptr) {
      for (int k = threadIdx.x; k < J.count; k += blockDim.x) J.dst[k] = J.src[k];
      continue;
    }
    for (int k = threadIdx.x; k < J.count; k += blockDim.x) {
      const int src = J.perm_off >= 0 ? perm[J.perm_off + k] : k;
      const double v = J.src != nullptr ? J.src[src] : 0.0;
      cd[J.dst_off + k] = v;
      cf[J.dst_off + k] = (float)v;
    }
  }
}

// grad[k] = sum_i w_i J[i][k] (with `data`: w_i = 2 (mean_i - data_i), and
// loss = sum_i (mean_i - data_i)^2 into *loss).  A block owns 64 columns;
// its 4 wavefronts take rows r = 4 t + wave (coalesced 64-column row
// segments), each lane sums its column over those rows in row order, and the
// four partial sums are added in wave order: a fixed order, so the result is
// bitwise reproducible.
__global__ void k_jacobian_apply(const double* __restrict__ jac, int64_t n_rows, int64_t ld, int64_t n_cols,
                                 const double* __restrict__ w, const pdd_node_stat_dev* __restrict__ stats,
                                 const double* __restrict__ data, double* __restrict__ grad,
                                 double* __restrict__ loss) {
  constexpr int kW = kBlock / kWave;
  __shared__ double part[kW][kWave];
  const int lane = (int)(threadIdx.x & (kWave - 1));
  const int wv = (int)(threadIdx.x / kWave);
  const int64_t col = (int64_t)blockIdx.x * kWave + lane;
  double acc = 0.0, lacc = 0.0;
  for (int64_t r = wv; r < n_rows; r += kW) {
    double wi;
    if (data != nullptr) {
      const double e = stats[r].mean - data[r];
      wi = 2.0 * e;
      lacc += e * e;
    } else {
      wi = w[r];
    }
    if (col < n_cols) acc += wi * jac[(size_t)r * ld + col];
  }
  part[wv][lane] = acc;
  __syncthreads();
  if (wv == 0 && col < n_cols) {
    double s = part[0][lane];
#pragma unroll
    for (int k = 1; k < kW; ++k) s += part[k][lane];
    grad[col] = s;
  }
  if (loss != nullptr && blockIdx.x == 0) {
    __syncthreads();
    part[wv][lane] = lacc;   // every lane of a wave holds the same partial loss
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = part[0][0];
#pragma unroll
      for (int k = 1; k < kW; ++k) s += part[k][0];
      *loss = s;
    }
  }
}

// Merges a second sample of node index[k] into the node's estimate: Chan's
// merge of the Welford triples, sums of the counts, and the Jacobian rows
// weighted by their path counts.  One block per merged node.
__global__ void k_merge_estimates(pdd_node_stat_dev* __restrict__ acc, double* __restrict__ acc_jac,
                                  int64_t acc_ld, const pdd_node_stat_dev* __restrict__ add,
                                  const double* __restrict__ add_jac, int64_t add_ld, int64_t n_params,
                                  const int64_t* __restrict__ index) {
  const int64_t k = blockIdx.x;
  const int64_t i = index[k];
  const pdd_node_stat_dev a = acc[i];
  const pdd_node_stat_dev b = add[k];
  const double na = (double)a.n, nb = (double)b.n;
  const double tot = na + nb;
  if (acc_jac != nullptr && add_jac != nullptr && tot > 0.0) {
    for (int64_t c = threadIdx.x; c < n_params; c += blockDim.x) {
      const double v = (na * acc_jac[(size_t)i * acc_ld + c] + nb * add_jac[(size_t)k * add_ld + c]) / tot;
      acc_jac[(size_t)i * acc_ld + c] = v;
    }
  }
  if (threadIdx.x == 0) {
    double n = na, m = a.mean, q = a.m2;
    chan_merge(n, m, q, nb, b.mean, b.m2);
    pdd_node_stat_dev r;
    r.mean = m; r.m2 = q; r.n = a.n + b.n; r.steps = a.steps + b.steps; r.censored = a.censored + b.censored;
    acc[i] = r;
  }
}

// var_i = m2_i / (n_i - 1) (0 for n_i < 2), se_i = sqrt(var_i / n_i).
__global__ void k_node_moments(const pdd_node_stat_dev* __restrict__ stats, int64_t n, double* __restrict__ var,
                               double* __restrict__ se) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const pdd_node_stat_dev s = stats[i];
  const double v = s.n > 1 ? s.m2 / (double)(s.n - 1) : 0.0;
  if (var != nullptr) var[i] = v;
  if (se != nullptr) se[i] = s.n > 0 ? sqrt(v / (double)s.n) : 0.0;
}

__global__ void k_fill_u32(uint32_t* p, int n, uint32_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_f64(double* p, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_walk_fwd(const WalkLaunch& L, hipStream_t st);
hipError_t launch_walk_adj_f32(const WalkLaunch& L, hipStream_t st);
hipError_t launch_walk_adj_f64(const WalkLaunch& L, hipStream_t st);

hipError_t launch_walk_wos(const WalkLaunch& L, hipStream_t st);

hipError_t launch_walk(const WalkLaunch& L, hipStream_t st) {
  if (L.spec != nullptr) {
    // same argument list as k_walk; the parameter block is passed by value
    const WorkItem* items = L.items;
    int n_items = L.n_items, grad_stride = L.grad_stride, refill = L.refill_groups;
    uint32_t* qhead = L.qhead;
    ItemStat* istat = L.istat;
    double* igrad = L.igrad;
    double* dump_phi = L.dump_phi;
    int64_t* dump_steps = L.dump_steps;
    const int64_t* dump_off = L.dump_off;
    void* args[] = {(void*)L.P, &items, &n_items, &qhead, &istat, &igrad, &grad_stride, &dump_phi, &dump_steps,
                    &dump_off, &refill};
    return hipModuleLaunchKernel(L.spec, (unsigned)L.grid, 1, 1, kBlock, 1, 1, 0, st, args, nullptr);
  }
  if (L.wos) return launch_walk_wos(L, st);
  if (!L.adjoint) return launch_walk_fwd(L, st);
  return L.fp32 ? launch_walk_adj_f32(L, st) : launch_walk_adj_f64(L, st);
}

hipError_t launch_finalize_nodes(const ItemStat* istat, const int64_t* first, int64_t n_nodes, const CallPtrs* cp,
                                 int64_t out_off, unsigned long long* counters, hipStream_t st) {
  const int64_t blocks = (n_nodes + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_finalize_nodes, dim3((unsigned)blocks), dim3(kBlock), 0, st, istat, first, n_nodes, cp,
                     out_off, counters);
  return hipGetLastError();
}

hipError_t launch_finalize_grad(const double* igrad, int stride, int n_cols, int n_items, const int32_t* slot_node,
                                const CallPtrs* cp, const double* inv_n, double* colsum, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize_grad, dim3(n_cols), dim3(kBlock), 0, st, igrad, stride, n_items, slot_node, cp,
                     inv_n, colsum);
  return hipGetLastError();
}

hipError_t launch_node_jacobian(const double* igrad, int stride, const int64_t* first, int64_t n_nodes,
                                const double* inv_n, const int32_t* colmap, int n_cols, const CallPtrs* cp,
                                int64_t jac_ld, hipStream_t st) {
  hipLaunchKernelGGL(k_node_jacobian, dim3((unsigned)n_nodes), dim3(kBlock), 0, st, igrad, stride, first, inv_n, colmap,
                     n_cols, cp, jac_ld);
  return hipGetLastError();
}

hipError_t launch_scatter_add(const double* src, const int32_t* map, int count, const CallPtrs* cp, int which,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_scatter_add, dim3((count + kBlock - 1) / kBlock), dim3(kBlock), 0, st, src, map, count, cp,
                     which);
  return hipGetLastError();
}

hipError_t launch_jacobian_apply(const double* jac, int64_t n_rows, int64_t ld, int64_t n_cols, const double* w,
                                 const void* stats, const double* data, double* grad, double* loss, hipStream_t st) {
  const int64_t blocks = (n_cols + kWave - 1) / kWave;
  hipLaunchKernelGGL(k_jacobian_apply, dim3((unsigned)(blocks > 0 ? blocks : 1)), dim3(kBlock), 0, st, jac, n_rows,
                     ld, n_cols, w, (const pdd_node_stat_dev*)stats, data, grad, loss);
  return hipGetLastError();
}

hipError_t launch_merge_estimates(void* acc, double* acc_jac, int64_t acc_ld, const void* add, const double* add_jac,
                                  int64_t add_ld, int64_t n_params, const int64_t* index, int64_t n_add,
                                  hipStream_t st) {
  hipLaunchKernelGGL(k_merge_estimates, dim3((unsigned)n_add), dim3(kBlock), 0, st, (pdd_node_stat_dev*)acc, acc_jac,
                     acc_ld, (const pdd_node_stat_dev*)add, add_jac, add_ld, n_params, index);
  return hipGetLastError();
}

hipError_t launch_node_moments(const void* stats, int64_t n, double* var, double* se, hipStream_t st) {
  const int64_t blocks = (n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_node_moments, dim3((unsigned)(blocks > 0 ? blocks : 1)), dim3(kBlock), 0, st,
                     (const pdd_node_stat_dev*)stats, n, var, se);
  return hipGetLastError();
}

hipError_t launch_stage(const StageJob* jobs, int n_jobs, const int32_t* perm, double* cd, float* cf,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_stage, dim3(1), dim3(kBlock), 0, st, jobs, n_jobs, perm, cd, cf);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, int n, uint32_t v, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_u32, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t st) {
  const int64_t blocks = (n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)(blocks > 0 ? blocks : 1)), dim3(kBlock), 0, st, p, n, v);
  return hipGetLastError();
}

}  // namespace pdd
