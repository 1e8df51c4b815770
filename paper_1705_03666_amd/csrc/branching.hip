// Branching-diffusion estimator (Sec. 3.1, eq. 3.1; marked form of Sec. 3.2).
//
// One tree per lane, simulated depth first: a particle (segment) lives an
// Exp(beta) time, moves by an exact Brownian increment sigma sqrt(delta) zeta
// (the driving process is Brownian motion, so no time stepping is needed),
// and either reaches T (leaf: the product picks up psi(X_T)) or branches into
// I ~ q children (the weight picks up alpha_I / q_I).  Pending siblings live
// on a per-lane stack in LDS (depth kLdsDepth) that spills to global memory
// for deep trees.  Finished lanes take the next tree index of their work item.
//
// A particle's random numbers are addressed by its label l (root 1, child i
// of l is B l + i): counter (l_lo, stream << 24 | attempt << 20 | blk << 16 |
// l_hi16, tree, point), stream 1 = lifetime and type uniforms, stream 2 =
// Gaussians, so the tree does not depend on traversal order or schedule.
// A tree exceeding max_segments particles (or a 48-bit label) is pruned and
// drawn again with attempt + 1; after 16 attempts it counts as censored with
// value 0.
#include <hip/hip_runtime.h>

#include "pdd_device.hpp"
#include "pdd_kernels.hpp"

namespace pdd {

// LDS stack depth per lane (entries of 24 B in FP32, 40 B in FP64).
template <typename R>
constexpr int lds_depth() { return sizeof(R) == 4 ? 8 : 4; }

template <typename R>
struct BrScalars;
template <>
struct BrScalars<float> {
  __device__ static float sigma(const BranchParams& P) { return P.sigmaf; }
  __device__ static float T(const BranchParams& P) { return P.Tf; }
  __device__ static float lifetime(const BranchParams& P, float u) {
    return -0.6931471805599453f * __builtin_amdgcn_logf(u) * __builtin_amdgcn_rcpf(P.betaf);
  }
};
template <>
struct BrScalars<double> {
  __device__ static double sigma(const BranchParams& P) { return P.sigma; }
  __device__ static double T(const BranchParams& P) { return P.T; }
  __device__ static double lifetime(const BranchParams& P, double u) { return -log(u) / P.beta; }
};

__device__ __forceinline__ float fsqrt(float v) { return __builtin_amdgcn_sqrtf(v); }
__device__ __forceinline__ double fsqrt(double v) { return sqrt(v); }

// lifetime and type uniforms (stream 1)
template <typename R, int LAYOUT>
__device__ __forceinline__ void br_uniforms(uint64_t label, int attempt, uint32_t tree, uint32_t point,
                                            uint32_t k0, uint32_t k1, R& ulife, R& utype) {
  uint32_t c0 = (uint32_t)label;
  uint32_t c1 = (1u << 24) | ((uint32_t)attempt << 20) | (uint32_t)((label >> 32) & 0xFFFFu);
  uint32_t c2 = tree, c3 = point;
  philox4x32_10(c0, c1, c2, c3, k0, k1);
  if constexpr (LAYOUT == RNG_QUAD24) {
    if constexpr (sizeof(R) == 4) {
      ulife = u24f(c0);
      utype = u24f(c1);
    } else {
      ulife = u24d(c0);
      utype = u24d(c1);
    }
  } else {
    ulife = (R)u52d(c0, c1);
    utype = (R)u52d(c2, c3);
  }
}

// first DIM Gaussians of stream 2
template <typename R, int DIM, int LAYOUT>
__device__ __forceinline__ void br_normals(uint64_t label, int attempt, uint32_t tree, uint32_t point, uint32_t k0,
                                           uint32_t k1, R* z) {
  using NZr = Normals<R, LAYOUT>;
  R tmp[4];
  const uint32_t base = (2u << 24) | ((uint32_t)attempt << 20) | (uint32_t)((label >> 32) & 0xFFFFu);
  NZr::gen((uint32_t)label, base, tree, point, k0, k1, tmp);
  if constexpr (NZr::kPerBlock == 2) {
    if constexpr (DIM > 2) NZr::gen((uint32_t)label, base | (1u << 16), tree, point, k0, k1, tmp + 2);
  }
#pragma unroll
  for (int k = 0; k < DIM; ++k) z[k] = tmp[k];
}

template <typename R, int DIM>
__device__ __forceinline__ R psi_value(const BranchParams& P, const R* x) {
  R v = (R)0;
  if (P.psi.n_terms > 0) v = terms_sum<R, DIM>(P.fac, P.cd, P.cf, P.psi, x);
  if (P.psi.poly_deg >= 0) v += poly_nested<R, DIM>(P.cd, P.cf, P.psi.poly_deg, P.psi.poly_off, x);
  return v;
}

template <typename R>
struct StackEntry {
  uint32_t lo, hi;
  R x[3];
  R t;
};

template <typename R, int DIM, int LAYOUT>
__global__ void __launch_bounds__(kBlock)
k_branch(const BranchParams P, const WorkItem* __restrict__ items, int n_items, uint32_t* __restrict__ qhead,
         ItemStat* __restrict__ istat, double* __restrict__ dump_val, int64_t* __restrict__ dump_segs,
         int64_t trees, StackEntry<R>* __restrict__ spill, int64_t spill_entries) {
  const int lane = (int)(threadIdx.x & (kWave - 1));
  const int wid = (int)(threadIdx.x / kWave);
  const int64_t glane = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t nlanes = (int64_t)gridDim.x * kBlock;
  constexpr int kLdsDepth = lds_depth<R>();
  __shared__ StackEntry<R> lds[kBlock / kWave][kLdsDepth][kWave];

  const uint32_t k0 = P.key0, k1 = P.key1;
  const R sigma = BrScalars<R>::sigma(P);
  const R Tend = BrScalars<R>::T(P);
  const uint64_t B = (uint64_t)P.label_base;

  for (;;) {
    const uint32_t it_idx = pop_item(qhead);
    if (it_idx >= (uint32_t)n_items) break;
    const WorkItem it = items[it_idx];
    const int point = it.node;
    const uint32_t pend = it.p0 + it.count;
    R x0[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) x0[k] = (R)P.points[(size_t)point * DIM + k];

    uint32_t tree = it.p0 + (uint32_t)lane;
    bool active = tree < pend;
    uint32_t cursor = it.p0 + (it.count < (uint32_t)kWave ? it.count : (uint32_t)kWave);

    // current segment and tree state
    uint64_t label = 1;
    R X[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) X[k] = x0[k];
    R tb = (R)0;
    double W = 1.0, prod = 1.0;
    int segs = 0, sp = 0, attempt = 0;

    double wn = 0.0, wmean = 0.0, wm2 = 0.0;
    int64_t lsegs = 0, lcens = 0, lredraw = 0;

    while (__any(active)) {
      bool done = false;
      double value = 0.0;
      if (active) {
        bool fail = false;
        ++segs;
        if (segs > P.max_segments) fail = true;
        if (!fail) {
          R ulife, utype, z[DIM];
          br_uniforms<R, LAYOUT>(label, attempt, tree, (uint32_t)point, k0, k1, ulife, utype);
          br_normals<R, DIM, LAYOUT>(label, attempt, tree, (uint32_t)point, k0, k1, z);
          const R E = BrScalars<R>::lifetime(P, ulife);
          const R rem = Tend - tb;
          const R delta = E < rem ? E : rem;
          const R sd = sigma * fsqrt(delta);
#pragma unroll
          for (int k = 0; k < DIM; ++k) X[k] = X[k] + sd * z[k];
          bool pop = false;
          if (E < rem) {
            // offspring count: smallest I with u < q_0 + ... + q_I (among q_I > 0)
            int I = 0;
            int last = 0;
            bool found = false;
#pragma unroll
            for (int k = 0; k < 5; ++k) {
              if (P.q[k] > 0.0) {
                last = k;
                const bool hit = sizeof(R) == 4 ? ((float)utype < P.qcumf[k]) : ((double)utype < P.qcum[k]);
                if (!found && hit) { I = k; found = true; }
              }
            }
            if (!found) I = last;
            double ratio = P.ratio[0];
#pragma unroll
            for (int k = 1; k < 5; ++k) if (I == k) ratio = P.ratio[k];
            W = W * ratio;
            if (I == 0) {
              pop = true;
            } else {
              const uint64_t first = B * label;
              if (label >= (1ull << 47) || first + (uint64_t)(I - 1) >= (1ull << 48) || sp + I - 1 > spill_entries + kLdsDepth) {
                fail = true;
              } else {
                const R tc = tb + E;
                for (int i = I - 1; i >= 1; --i) {
                  StackEntry<R> s;
                  const uint64_t cl = first + (uint64_t)i;
                  s.lo = (uint32_t)cl;
                  s.hi = (uint32_t)(cl >> 32);
#pragma unroll
                  for (int k = 0; k < 3; ++k) s.x[k] = k < DIM ? X[k] : (R)0;
                  s.t = tc;
                  if (sp < kLdsDepth) lds[wid][sp][lane] = s;
                  else spill[(int64_t)(sp - kLdsDepth) * nlanes + glane] = s;
                  ++sp;
                }
                label = first;
                tb = tc;
              }
            }
          } else {
            prod = prod * (double)psi_value<R, DIM>(P, X);
            pop = true;
          }
          if (!fail && pop) {
            if (sp == 0) {
              done = true;
              value = prod * W;
            } else {
              --sp;
              const StackEntry<R> s = sp < kLdsDepth ? lds[wid][sp][lane]
                                                     : spill[(int64_t)(sp - kLdsDepth) * nlanes + glane];
              label = (uint64_t)s.lo | ((uint64_t)s.hi << 32);
#pragma unroll
              for (int k = 0; k < DIM; ++k) X[k] = s.x[k];
              tb = s.t;
            }
          }
        }
        if (fail) {
          ++lredraw;
          ++attempt;
          if (attempt >= 16) {
            done = true;
            value = 0.0;
            ++lcens;
          } else {
            label = 1;
#pragma unroll
            for (int k = 0; k < DIM; ++k) X[k] = x0[k];
            tb = (R)0;
            W = 1.0;
            prod = 1.0;
            segs = 0;
            sp = 0;
          }
        }
        if (done) {
          wn += 1.0;
          const double d1 = value - wmean;
          wmean += d1 / wn;
          wm2 += d1 * (value - wmean);
          lsegs += segs;
          if (dump_val != nullptr) {
            const int64_t o = (int64_t)point * trees + (int64_t)tree;
            dump_val[o] = value;
            if (dump_segs != nullptr) dump_segs[o] = segs;
          }
        }
      }
      // refill
      const uint64_t dmask = ballot(done);
      if (dmask != 0) {
        const uint32_t nt = cursor + (uint32_t)lane_rank(dmask);
        cursor += (uint32_t)__popcll(dmask);
        if (done) {
          if (nt < pend) {
            tree = nt;
            label = 1;
#pragma unroll
            for (int k = 0; k < DIM; ++k) X[k] = x0[k];
            tb = (R)0;
            W = 1.0;
            prod = 1.0;
            segs = 0;
            sp = 0;
            attempt = 0;
          } else {
            active = false;
          }
        }
      }
    }

    wave_welford(wn, wmean, wm2);
    lsegs = wave_sum(lsegs);
    lcens = wave_sum(lcens);
    lredraw = wave_sum(lredraw);
    if (lane == 0) {
      ItemStat st;
      st.mean = wmean;
      st.m2 = wm2;
      st.n = (int64_t)wn;
      st.steps = lsegs;
      st.censored = lcens;
      st.redrawn = lredraw;
      istat[it.slot] = st;
    }
  }
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
  if (L.fp32) return launch_branch_t<float, RNG_QUAD24>(L, st);
  if (L.layout == RNG_QUAD24) return launch_branch_t<double, RNG_QUAD24>(L, st);
  return launch_branch_t<double, RNG_PAIR52>(L, st);
}

}  // namespace pdd
