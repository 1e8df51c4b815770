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
//
// psi and g are evaluated through a policy: TablePsi reads the staged term
// table (any problem); the library can also compile these kernels at run time
// with a policy that has one problem's factor structure written in (see
// specialize.cpp), which evaluates the same operations in the same order.
#pragma once
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#endif

#include "pdd_device.hpp"

namespace pdd {

// LDS stack depth per lane (entries of 24 B in FP32, 40 B in FP64); deeper
// entries go to the per-lane spill area in global memory.  Six FP32 entries
// keep a 256-thread block at 37 KB of LDS, so four blocks fit a CU (eight
// entries allowed three: measured 13% slower on C6, 6-12% on C4 / C7; three
// entries and six blocks per CU: C4 1% slower, C7 slower).
template <typename R>
constexpr int lds_depth() { return sizeof(R) == 4 ? 6 : 4; }

// FP32 kernels are built for four waves per SIMD (at most 128 VGPRs).
template <typename R>
constexpr int branch_min_waves() { return sizeof(R) == 4 ? 4 : 1; }

template <typename R>
struct BrScalars;
template <>
struct BrScalars<float> {
  __device__ static float sigma(const BranchParams& P) { return P.sigmaf; }
  __device__ static float T(const BranchParams& P) { return P.Tf; }
  __device__ static float lifetime(const BranchParams& P, float u) {
    return -0.6931471805599453f * __builtin_amdgcn_logf(u) * P.inv_betaf;
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
  // opaque copies of the key: the round keys are rebuilt with scalar adds at
  // each use instead of holding twenty scalar registers through the loop
  uint32_t ka = k0, kb = k1;
  asm volatile("" : "+s"(ka), "+s"(kb));
  philox4x32_10(c0, c1, c2, c3, ka, kb);
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
  uint32_t ka = k0, kb = k1;
  asm volatile("" : "+s"(ka), "+s"(kb));
  NZr::gen((uint32_t)label, base, tree, point, ka, kb, tmp);
  if constexpr (NZr::kPerBlock == 2) {
    if constexpr (DIM > 2) {
      uint32_t kc = k0, kd = k1;
      asm volatile("" : "+s"(kc), "+s"(kd));
      NZr::gen((uint32_t)label, base | (1u << 16), tree, point, kc, kd, tmp + 2);
    }
  }
#pragma unroll
  for (int k = 0; k < DIM; ++k) z[k] = tmp[k];
}

// Both Philox blocks of an FP32 segment (stream 1: lifetime and type
// uniforms; stream 2: the Gaussians) computed round by round side by side:
// the same two blocks as br_uniforms and br_normals, with four independent
// products per round instead of two, and one key schedule for both (C4
// 3.45 -> 3.37 ms, C7 2.09 -> 2.06 ms; the trees are bitwise unchanged).
__device__ __forceinline__ void philox_pair(uint32_t* a, uint32_t* b, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t pa0 = (uint64_t)0xD2511F53u * (uint64_t)a[0];
    const uint64_t pa1 = (uint64_t)0xCD9E8D57u * (uint64_t)a[2];
    const uint64_t pb0 = (uint64_t)0xD2511F53u * (uint64_t)b[0];
    const uint64_t pb1 = (uint64_t)0xCD9E8D57u * (uint64_t)b[2];
    const uint32_t na0 = xor3((uint32_t)(pa1 >> 32), a[1], k0);
    const uint32_t na2 = xor3((uint32_t)(pa0 >> 32), a[3], k1);
    const uint32_t nb0 = xor3((uint32_t)(pb1 >> 32), b[1], k0);
    const uint32_t nb2 = xor3((uint32_t)(pb0 >> 32), b[3], k1);
    a[1] = (uint32_t)pa1;
    a[3] = (uint32_t)pa0;
    a[0] = na0;
    a[2] = na2;
    b[1] = (uint32_t)pb1;
    b[3] = (uint32_t)pb0;
    b[0] = nb0;
    b[2] = nb2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// A segment's lifetime and type uniforms and its first DIM Gaussians.
template <typename R, int DIM, int LAYOUT>
__device__ __forceinline__ void br_draws(uint64_t label, int attempt, uint32_t tree, uint32_t point, uint32_t k0,
                                         uint32_t k1, R& ulife, R& utype, R* z) {
  if constexpr (sizeof(R) == 4 && LAYOUT == RNG_QUAD24) {
    const uint32_t hi = ((uint32_t)attempt << 20) | (uint32_t)((label >> 32) & 0xFFFFu);
    uint32_t a[4] = {(uint32_t)label, (1u << 24) | hi, tree, point};
    uint32_t b[4] = {(uint32_t)label, (2u << 24) | hi, tree, point};
    uint32_t ka = k0, kb = k1;
    asm volatile("" : "+s"(ka), "+s"(kb));
    philox_pair(a, b, ka, kb);
    ulife = u24f(a[0]);
    utype = u24f(a[1]);
    float t[4];
    box_muller_f(u24f(b[0]), u24f(b[1]), t[0], t[1]);
    box_muller_f(u24f(b[2]), u24f(b[3]), t[2], t[3]);
#pragma unroll
    for (int k = 0; k < DIM; ++k) z[k] = t[k];
  } else {
    br_uniforms<R, LAYOUT>(label, attempt, tree, point, k0, k1, ulife, utype);
    br_normals<R, DIM, LAYOUT>(label, attempt, tree, point, k0, k1, z);
  }
}

// Offspring class of a branching particle with type uniform u: the index j
// into the compact law (class size P.cls[j], mark P.mark[j]), i.e. the number
// of class thresholds at or below u -- the first class whose cumulative
// probability exceeds u, the last class for larger u.
template <typename R>
__device__ __forceinline__ int offspring_class(const BranchParams& P, R u) {
  int j = 0;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const bool ge = sizeof(R) == 4 ? ((float)u >= P.thrf[m]) : ((double)u >= P.thr[m]);
    j += ge ? 1 : 0;
  }
  return j;
}

__device__ __forceinline__ int class_size(const BranchParams& P, int j) {
  int I = P.cls[0];
#pragma unroll
  for (int m = 1; m < 5; ++m) I = j == m ? P.cls[m] : I;
  return I;
}

__device__ __forceinline__ double class_mark(const BranchParams& P, int j) {
  double r = P.mark[0];
#pragma unroll
  for (int m = 1; m < 5; ++m) r = j == m ? P.mark[m] : r;
  return r;
}

// psi and g from the staged term table: the sum of the generic terms, then
// the dense polynomial part.  g takes the boundary point xp and the time
// argument ts as coordinates 0..DIM-1 and DIM of its terms; its polynomial
// part reads xp only.
struct TablePsi {
  template <typename R, int DIM>
  __device__ static __forceinline__ R psi(const BranchParams& P, const R* x) {
    R v = (R)0;
    if (P.psi.n_terms > 0) v = terms_sum<R, DIM>(P.fac, P.cd, P.cf, P.psi, x);
    if (P.psi.poly_deg >= 0) v += poly_nested<R, DIM>(P.cd, P.cf, P.psi.poly_deg, P.psi.poly_off, x);
    return v;
  }
  template <typename R, int DIM>
  __device__ static __forceinline__ R g(const BranchParams& P, const BranchBoundary& B, const R* xp, R ts) {
    R xs[DIM + 1];
#pragma unroll
    for (int k = 0; k < DIM; ++k) xs[k] = xp[k];
    xs[DIM] = ts;
    R v = (R)0;
    if (B.g.n_terms > 0) v = terms_sum<R, DIM + 1>(P.fac, P.cd, P.cf, B.g, xs);
    if (B.g.poly_deg >= 0) v += poly_nested<R, DIM>(P.cd, P.cf, B.g.poly_deg, B.g.poly_off, xp);
    return v;
  }
};

template <typename R>
struct StackEntry {
  uint32_t lo, hi;
  R x[3];
  R t;
};

template <typename R, int DIM, int LAYOUT, typename PSI = TablePsi>
__global__ void __launch_bounds__(kBlock, (branch_min_waves<R>()))
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

    // per-lane accumulation of the finished trees' values as shifted sums
    // (count, shift = the lane's first value, sums of v - shift and of its
    // square): no division per tree; converted to a Welford triple and
    // merged across the wavefront once per item
    double wn = 0.0, wk = 0.0, ws1 = 0.0, ws2 = 0.0;
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
          br_draws<R, DIM, LAYOUT>(label, attempt, tree, (uint32_t)point, k0, k1, ulife, utype, z);
          const R E = BrScalars<R>::lifetime(P, ulife);
          const R rem = Tend - tb;
          const R delta = E < rem ? E : rem;
          const R sd = sigma * fsqrt(delta);
#pragma unroll
          for (int k = 0; k < DIM; ++k) X[k] = X[k] + sd * z[k];
          bool pop = false;
          if (E < rem) {
            // offspring count: smallest I with u < q_0 + ... + q_I (among q_I > 0)
            const int jc = offspring_class<R>(P, utype);
            const int I = class_size(P, jc);
            W = W * class_mark(P, jc);
            if (I == 0) {
              pop = true;
            } else {
              const uint64_t first = B * label;
              if (label >= (1ull << 47) || first + (uint64_t)(I - 1) >= (1ull << 48) ||
                  sp + I - 1 > spill_entries + kLdsDepth) {
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
            prod = prod * (double)PSI::template psi<R, DIM>(P, X);
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
          wk = wn == 0.0 ? value : wk;
          const double dv = value - wk;
          wn += 1.0;
          ws1 += dv;
          ws2 += dv * dv;
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

    double wmean = 0.0, wm2 = 0.0;
    if (wn > 0.0) {
      const double a = ws1 / wn;
      wmean = wk + a;
      wm2 = ws2 - ws1 * a;
      wm2 = wm2 > 0.0 ? wm2 : 0.0;
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

// ---------------------------------------------------------------------------
// Branching with a Dirichlet boundary, several output times (eq. 3.2,
// Algorithm 3.1).  One tree per lane, depth first as above; a particle now
// moves by exact Brownian increments over sub-steps that end at
// min(s + dt, its death time, the last output time, the next output time),
// and is tested against the boundary after each sub-step except the one that
// ends at its death (the children are tested at their birth instead; a test
// there would anticipate the death time).  With the boundary correction the
// test after a sub-step of length h uses D shrunk by c0 sigma sqrt(h).  A
// particle found outside is projected and stopped: every output time t_i >= s picks up g(P X, t_i - s).
// A particle inside at an output time t_k multiplies factor k by psi(X); a
// branching at time s multiplies every factor with t_i > s by alpha_I / q_I.
// The per-tree factors are FP64 products; a finished tree enters the
// wavefront's FP64 Welford triple of every output time (kept in LDS, lanes
// in order).  Lanes run sub-steps in rounds over windows of their Gaussians
// (bvp_round) and stop at their first event (output time, stop, death, end),
// which is handled after the round, so the rare event code is not
// interleaved with every sub-step.
// The statistics' step count is the number of particle sub-steps.
//
// Gaussians: number n DIM + c of a particle (sub-step n, coordinate c) is
// slot (n DIM + c) mod m of Philox block j = (n DIM + c) / m (m normals per
// block), counter (label_lo, 5 << 28 | attempt << 24 | label_hi16 << 8 |
// j >> 8, tree, point | (j & 255) << 24).
template <typename R>
struct BvScalars;
template <>
struct BvScalars<float> {
  __device__ static float dt(const BranchBoundary& B) { return B.dtf; }
  __device__ static float t(const BranchBoundary& B, int i) { return B.timesf[i]; }
  __device__ static float shift(const BranchBoundary& B) { return B.shiftf; }
};
template <>
struct BvScalars<double> {
  __device__ static double dt(const BranchBoundary& B) { return B.dt; }
  __device__ static double t(const BranchBoundary& B, int i) { return B.times[i]; }
  __device__ static double shift(const BranchBoundary& B) { return B.shift; }
};

template <typename R>
__device__ __forceinline__ Dom<R> bvp_dom(const BranchBoundary& B);
template <>
__device__ __forceinline__ Dom<float> bvp_dom<float>(const BranchBoundary& B) {
  Dom<float> D;
  D.kind = B.dom_kind;
  for (int k = 0; k < 3; ++k) { D.lo[k] = B.lof[k]; D.hi[k] = B.hif[k]; D.ctr[k] = B.ctrf[k]; }
  D.rad = B.radf;
  D.rad2 = B.rad2f;
  return D;
}
template <>
__device__ __forceinline__ Dom<double> bvp_dom<double>(const BranchBoundary& B) {
  Dom<double> D;
  D.kind = B.dom_kind;
  for (int k = 0; k < 3; ++k) { D.lo[k] = B.lo[k]; D.hi[k] = B.hi[k]; D.ctr[k] = B.ctr[k]; }
  D.rad = B.rad;
  D.rad2 = B.rad2;
  return D;
}

// Event batching: lanes with an event wait until this many have one (or the
// conditions in k_branch_bvp), so the event code runs for several at once.
constexpr int kEvBatch = 64;
constexpr int kEvWait = 32;

// Sub-steps per round: the Gaussians of a particle are taken in windows of
// kW = steps * DIM numbers, a whole number of Philox blocks (1-D and 2-D: two
// blocks of four; 3-D: three), so every lane of a round draws the same kNB
// blocks of its own window and finds its Gaussians at fixed slots.
template <int DIM>
constexpr int bvp_round_steps() { return DIM == 1 ? 16 : (DIM == 2 ? 8 : 4); }

// One round of sub-steps over each stepping lane's current window of
// Gaussians (window gidx / kW): a lane whose next Gaussian is number o DIM of
// the window takes sub-steps o, o + 1, .. until its first event or the end of
// the window.  A sub-step ends at min(s + dt, lim), lim = min(end of stepping,
// next output time); the particle is tested against D shrunk by shift sd
// unless the sub-step ends at its death (dlim: lim is the death time, so a
// sub-step ending at lim is the death).  Predicated, without branches:
// `stepping` is cleared at the first event, `stopped` set when that event is
// a boundary stop.  KIND is the domain kind and SHIFT whether shift != 0
// (both uniform over the launch).  In FP32 the uniform parameters are copied
// into vector registers first, so the instructions that read them can share
// an issue slot.
template <typename R, int DIM, int LAYOUT, int KIND, bool SHIFT>
__device__ __forceinline__ void bvp_round(const Dom<R>& D, R sigma, R dt, R shift, uint64_t label, int attempt,
                                          uint32_t tree, uint32_t point, uint32_t k0, uint32_t k1, R lim, bool dlim,
                                          R* X, R& s, uint32_t& gidx, bool& stepping, bool& stopped, int& nsub) {
  using NZr = Normals<R, LAYOUT>;
  constexpr int kPer = NZr::kPerBlock;
  constexpr int kSub = bvp_round_steps<DIM>();
  constexpr int kW = kSub * DIM;
  constexpr int kNB = kW / kPer;
  static_assert(kW % kPer == 0, "a window is a whole number of Philox blocks");
  R zb[kW];
  const uint32_t w = gidx / (uint32_t)kW;
  const int o = (int)((gidx % (uint32_t)kW) / (uint32_t)DIM);
#pragma unroll
  for (int b = 0; b < kNB; ++b) {
    const uint32_t j = w * (uint32_t)kNB + (uint32_t)b;
    const uint32_t c0 = (uint32_t)label;
    const uint32_t c1 = (5u << 28) | ((uint32_t)attempt << 24) | ((uint32_t)((label >> 32) & 0xFFFFu) << 8) |
                        ((j >> 8) & 0xFFu);
    const uint32_t c3 = (point & 0xFFFFFFu) | ((j & 0xFFu) << 24);
    uint32_t ka = k0, kb = k1;
    asm volatile("" : "+s"(ka), "+s"(kb));
    NZr::gen(c0, c1, tree, c3, ka, kb, &zb[b * kPer]);
  }
  R lo[DIM], hi[DIM], ctr[DIM], rad = D.rad;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    lo[k] = D.lo[k];
    hi[k] = D.hi[k];
    ctr[k] = D.ctr[k];
  }
  if constexpr (sizeof(R) == 4) {
    asm volatile("" : "+v"(sigma), "+v"(dt), "+v"(shift));
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      if constexpr (KIND == DOM_BOX) asm volatile("" : "+v"(lo[k]), "+v"(hi[k]));
      if constexpr (KIND == DOM_BALL) asm volatile("" : "+v"(ctr[k]));
    }
    if constexpr (KIND == DOM_BALL) asm volatile("" : "+v"(rad));
  }
  int n = 0;
#pragma unroll
  for (int q = 0; q < kSub; ++q) {
    const bool st = stepping && o <= q;
    const R sn = fmin(s + dt, lim);
    const R sd = sigma * fsqrt(sn - s);
    R Xn[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) Xn[k] = X[k] + sd * zb[q * DIM + k];
    bool out = false;
    if constexpr (KIND == DOM_BOX) {
      bool in = true;
      if constexpr (SHIFT) {
        const R delta = shift * sd;
#pragma unroll
        for (int k = 0; k < DIM; ++k) in = in && (Xn[k] > lo[k] + delta) && (Xn[k] < hi[k] - delta);
      } else {
#pragma unroll
        for (int k = 0; k < DIM; ++k) in = in && (Xn[k] > lo[k]) && (Xn[k] < hi[k]);
      }
      out = !in;
    } else if constexpr (KIND == DOM_BALL) {
      R r2 = (R)0;
#pragma unroll
      for (int k = 0; k < DIM; ++k) {
        const R d = Xn[k] - ctr[k];
        r2 += d * d;
      }
      R rs = rad;
      if constexpr (SHIFT) {
        rs = rad - shift * sd;
        rs = rs > (R)0 ? rs : (R)0;
      }
      out = !(r2 < rs * rs);
    }
    const bool at = !(sn < lim);
    const bool stop = out && !(dlim && at);
#pragma unroll
    for (int k = 0; k < DIM; ++k) X[k] = st ? Xn[k] : X[k];
    s = st ? sn : s;
    n += st ? 1 : 0;
    stopped = stopped || (st && stop);
    stepping = stepping && !(st && (stop || at));
  }
  gidx += (uint32_t)(n * DIM);
  nsub += n;
}

// Boundary stops of several lanes at once: every lane with `need` multiplies
// Pt[i] by g(xp, t_i - s0) for each output time index f <= i < nt, f the
// first with t_i >= s0.  The (lane, time) pairs are dealt out one per lane,
// 64 per pass, through cross-lane reads, so a batch of stops costs about one
// evaluation of g per pass instead of one per output time; every factor is
// still the single product Pt[i] * g, so results do not change.  All lanes
// of the wavefront must call it.  `tms` holds the output times.
template <typename R, int DIM, typename PSI>
__device__ __forceinline__ void stop_products(bool need, const R* xp, R s0, double* Pt, const BranchParams& P,
                                              const BranchBoundary& BB, const R* tms, int nt, int lane) {
  if (!__any(need)) return;
  int f = nt;
#pragma unroll
  for (int i = kMaxTimes - 1; i >= 0; --i)
    if (i < nt && tms[i] >= s0) f = i;
  const int c = need ? nt - f : 0;
  int incl = c;   // inclusive prefix sum of c over the lanes
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int v = __shfl_up(incl, (unsigned)d);
    if (lane >= d) incl += v;
  }
  const int off = incl - c;
  const int total = __shfl(incl, kWave - 1);
  for (int base = 0; base < total; base += kWave) {
    const int g = base + lane;
    int l = 0;   // the lane whose pairs hold g: the first with incl > g
#pragma unroll
    for (int step = kWave / 2; step > 0; step >>= 1) {
      const int v = __shfl(incl, l + step - 1);
      if (v <= g) l += step;
    }
    l = l < kWave ? l : kWave - 1;
    R xs[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) xs[k] = __shfl(xp[k], l);
    const R sl = __shfl(s0, l);
    const int i = __shfl(f, l) + (g - __shfl(off, l));
    double r = 1.0;
    if (g < total) r = (double)PSI::template g<R, DIM>(P, BB, xs, tms[i] - sl);
#pragma unroll
    for (int i2 = 0; i2 < kMaxTimes; ++i2) {
      const int src = off + (i2 - f) - base;
      const double v = __shfl(r, src >= 0 && src < kWave ? src : 0);
      if (need && i2 >= f && i2 < nt && src >= 0 && src < kWave) Pt[i2] *= v;
    }
  }
}

// Events of a particle found at the end of a sub-step.
enum : int { EV_OUT = 1, EV_STOP = 2, EV_DEATH = 4, EV_END = 8 };

template <typename R, int DIM, int LAYOUT, typename PSI = TablePsi>
__global__ void __launch_bounds__(kBlock, (branch_min_waves<R>()))
k_branch_bvp(const BranchParams P, const BranchBoundary BB, const WorkItem* __restrict__ items, int n_items,
             uint32_t* __restrict__ qhead, ItemStat* __restrict__ istat, double* __restrict__ dump_val,
             int64_t* __restrict__ dump_segs, int64_t trees, StackEntry<R>* __restrict__ spill,
             int64_t spill_entries) {
  const int lane = (int)(threadIdx.x & (kWave - 1));
  const int wid = (int)(threadIdx.x / kWave);
  const int64_t glane = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t nlanes = (int64_t)gridDim.x * kBlock;
  constexpr int kLdsDepth = lds_depth<R>();
  __shared__ StackEntry<R> lds[kBlock / kWave][kLdsDepth][kWave];
  // per wavefront and output time i: shifted sums of the finished trees'
  // values (sum of v - K_i, sum of (v - K_i)^2, K_i = the first tree's
  // value), lane i updating time i; plus the tree count and a staging row
  // through which a finished tree hands its values to those lanes
  __shared__ double wst[kBlock / kWave][3 * kMaxTimes + 1];
  __shared__ double wrow[kBlock / kWave][kMaxTimes];
  // the output times, for lanes that index them at run time
  __shared__ R tms[kMaxTimes];
  if (threadIdx.x < (unsigned)kMaxTimes) tms[threadIdx.x] = BvScalars<R>::t(BB, (int)threadIdx.x);
  __syncthreads();

  const uint32_t k0 = P.key0, k1 = P.key1;
  const R sigma = BrScalars<R>::sigma(P);
  const R dt = BvScalars<R>::dt(BB);
  const R shift = BvScalars<R>::shift(BB);
  const int nt = BB.n_times;
  const R tend = BvScalars<R>::t(BB, nt - 1);
  const bool bounded = BB.dom_kind != DOM_FREE;
  const Dom<R> D = bvp_dom<R>(BB);
  const uint64_t B = (uint64_t)P.label_base;
  double* const W = &wst[wid][0];

  for (;;) {
    const uint32_t it_idx = pop_item(qhead);
    if (it_idx >= (uint32_t)n_items) break;
    const WorkItem it = items[it_idx];
    const int point = it.node;
    const uint32_t pend = it.p0 + it.count;
    R x0[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) x0[k] = (R)P.points[(size_t)point * DIM + k];
    // output times at 0 take psi at the start point when it is inside
    const bool x0_in = !bounded || inside<R, DIM>(D, x0);
    const double psi0 = x0_in ? (double)PSI::template psi<R, DIM>(P, x0) : 1.0;
    __builtin_amdgcn_wave_barrier();
    if (lane < 3 * kMaxTimes + 1) W[lane] = 0.0;
    __builtin_amdgcn_wave_barrier();

    uint32_t tree = it.p0 + (uint32_t)lane;
    bool active = tree < pend;
    uint32_t cursor = it.p0 + (it.count < (uint32_t)kWave ? it.count : (uint32_t)kWave);

    // particle state: position, time, death time, end of its stepping
    // (min(death, last output time)), next output index and time
    uint64_t label = 1;
    R X[DIM];
    R s = (R)0, sdeath = (R)0, send = (R)0, tk = (R)0, utype = (R)0;
    uint32_t gidx = 0;
    int kout = 0;
    bool fresh = true;
    // tree state
    double Pt[kMaxTimes];
    int segs = 0, sp = 0, attempt = 0;
    auto start_tree = [&]() {
      label = 1;
#pragma unroll
      for (int k = 0; k < DIM; ++k) X[k] = x0[k];
      s = (R)0;
      fresh = true;
      segs = 0;
      sp = 0;
#pragma unroll
      for (int i = 0; i < kMaxTimes; ++i) Pt[i] = (i < nt && !(BvScalars<R>::t(BB, i) > (R)0)) ? psi0 : 1.0;
    };
    start_tree();
    int64_t lsub = 0, lcens = 0, lredraw = 0;
    // a lane's pending event (0: none); rounds since events were last handled
    int ev = 0;
    int since = 0;

    while (__any(active)) {
      bool done = false, censored = false, fail = false;
      // ---- births: test at birth, lifetime and type (a lane whose particle
      // is stopped at birth pops and may meet another birth: loop)
      for (;;) {
        const bool need = active && fresh && !done && !fail;
        if (!__any(need)) break;
        bool stop0 = false;
        if (need) {
          ++segs;
          if (segs > P.max_segments) {
            fail = true;
          } else if (bounded && !inside<R, DIM>(D, X)) {
            stop0 = true;
          } else {
            R ulife;
            br_uniforms<R, LAYOUT>(label, attempt, tree, (uint32_t)point, k0, k1, ulife, utype);
            sdeath = s + BrScalars<R>::lifetime(P, ulife);
            send = sdeath < tend ? sdeath : tend;
            kout = 0;
            tk = tend;
#pragma unroll
            for (int i = kMaxTimes - 1; i >= 0; --i) {
              const R ti = BvScalars<R>::t(BB, i);
              if (i < nt && ti > s) { kout = i; tk = ti; }
            }
            if (!(tk > s)) kout = nt;   // no output time after s
            gidx = 0;
            fresh = false;
          }
        }
        {
          // born outside: stopped at its birth time
          R xp[3] = {(R)0, (R)0, (R)0};
          if (stop0) project<R, DIM>(D, X, xp);
          stop_products<R, DIM, PSI>(stop0, xp, s, Pt, P, BB, tms, nt, lane);
        }
        if (need) {
          if (stop0) {
            if (sp == 0) {
              done = true;
            } else {
              --sp;
              const StackEntry<R> e = sp < kLdsDepth ? lds[wid][sp][lane]
                                                     : spill[(int64_t)(sp - kLdsDepth) * nlanes + glane];
              label = (uint64_t)e.lo | ((uint64_t)e.hi << 32);
#pragma unroll
              for (int k = 0; k < DIM; ++k) X[k] = e.x[k];
              s = e.t;
            }
          }
        }
      }
      // ---- a round of sub-steps; a lane stops at its first event, whose kind
      // follows from where it stopped
      bool stepping = active && !fresh && !done && !fail && ev == 0;
      if (stepping && !(s < send)) {   // nothing left to step (a last output time of 0)
        ev = EV_END;
        stepping = false;
      }
      const bool stepped = stepping;
      bool stopped = false;
      {
        R lim = send;
        if (kout < nt && tk < lim) lim = tk;
        const bool dcand = sdeath < tend;
        // the sub-step that ends at lim ends at the death: no boundary test
        const bool dlim = dcand && lim == sdeath;
        int nsub = 0;
#define PDD_BVP_ROUND(KIND, SHIFT)                                                                              \
  bvp_round<R, DIM, LAYOUT, KIND, SHIFT>(D, sigma, dt, shift, label, attempt, tree, (uint32_t)point, k0, k1, lim, \
                                         dlim, X, s, gidx, stepping, stopped, nsub)
        if (D.kind == DOM_BOX) {
          if (shift != (R)0) PDD_BVP_ROUND(DOM_BOX, true);
          else PDD_BVP_ROUND(DOM_BOX, false);
        } else if (D.kind == DOM_BALL) {
          if (shift != (R)0) PDD_BVP_ROUND(DOM_BALL, true);
          else PDD_BVP_ROUND(DOM_BALL, false);
        } else {
          PDD_BVP_ROUND(DOM_FREE, false);
        }
#undef PDD_BVP_ROUND
        lsub += nsub;
        if (stepped && !stepping) {
          if (stopped) {
            ev = EV_STOP;
          } else {   // s == lim
            if (kout < nt && s == tk) ev |= EV_OUT;
            if (!(s < send)) ev |= (dcand && s == sdeath) ? EV_DEATH : EV_END;
          }
        }
      }
      // ---- events, handled for several lanes at once: a lane with an event
      // waits (takes no sub-steps) until kEvBatch lanes have one, every active
      // lane has one, kEvWait rounds have passed, or a tree has ended
      const uint64_t pmask = ballot(ev != 0);
      const bool handle = __popcll(pmask) >= kEvBatch || pmask == ballot(active) || since >= kEvWait ||
                          __any(done || fail);
      since = handle ? 0 : since + 1;
      if (handle) {
        {
          // projected onto the boundary and stopped at time s
          const bool stopnow = (ev & EV_STOP) != 0;
          R xp[3] = {(R)0, (R)0, (R)0};
          if (stopnow) project<R, DIM>(D, X, xp);
          stop_products<R, DIM, PSI>(stopnow, xp, s, Pt, P, BB, tms, nt, lane);
        }
        if (ev != 0) {
          bool pop = false;
          if (ev & EV_OUT) {
            const double pv = (double)PSI::template psi<R, DIM>(P, X);
#pragma unroll
            for (int i = 0; i < kMaxTimes; ++i)
              if (i == kout) Pt[i] *= pv;
            ++kout;
#pragma unroll
            for (int i = 0; i < kMaxTimes; ++i)
              if (i == kout) tk = BvScalars<R>::t(BB, i);
          }
          if (ev & EV_STOP) {
            pop = true;
          } else if (ev & EV_END) {
            pop = true;   // reached the last output time
          } else if (ev & EV_DEATH) {
            // offspring count: smallest I with u < q_0 + ... + q_I (among q_I > 0)
            const int jc = offspring_class<R>(P, utype);
            const int I = class_size(P, jc);
            const double ratio = class_mark(P, jc);
            if (ratio != 1.0) {
#pragma unroll
              for (int i = 0; i < kMaxTimes; ++i)
                if (i < nt && BvScalars<R>::t(BB, i) > sdeath) Pt[i] *= ratio;
            }
            if (I == 0) {
              pop = true;
            } else {
              const uint64_t first = B * label;
              if (label >= (1ull << 47) || first + (uint64_t)(I - 1) >= (1ull << 48) ||
                  sp + I - 1 > spill_entries + kLdsDepth) {
                fail = true;
              } else {
                for (int i = I - 1; i >= 1; --i) {
                  StackEntry<R> e;
                  const uint64_t cl = first + (uint64_t)i;
                  e.lo = (uint32_t)cl;
                  e.hi = (uint32_t)(cl >> 32);
#pragma unroll
                  for (int k = 0; k < 3; ++k) e.x[k] = k < DIM ? X[k] : (R)0;
                  e.t = sdeath;
                  if (sp < kLdsDepth) lds[wid][sp][lane] = e;
                  else spill[(int64_t)(sp - kLdsDepth) * nlanes + glane] = e;
                  ++sp;
                }
                label = first;
                s = sdeath;
                fresh = true;
              }
            }
          }
          if (pop && !fail) {
            if (sp == 0) {
              done = true;
            } else {
              --sp;
              const StackEntry<R> e = sp < kLdsDepth ? lds[wid][sp][lane]
                                                     : spill[(int64_t)(sp - kLdsDepth) * nlanes + glane];
              label = (uint64_t)e.lo | ((uint64_t)e.hi << 32);
#pragma unroll
              for (int k = 0; k < DIM; ++k) X[k] = e.x[k];
              s = e.t;
              fresh = true;
            }
          }
        }
        if (fail) {
          ++lredraw;
          ++attempt;
          if (attempt >= 16) {
            done = true;
            censored = true;
            ++lcens;
          } else {
            start_tree();
          }
        }
        if (done) {
          if (censored) {
#pragma unroll
            for (int i = 0; i < kMaxTimes; ++i) Pt[i] = 0.0;
          }
          if (dump_val != nullptr) {
            const int64_t o = ((int64_t)point * trees + (int64_t)tree) * nt;
#pragma unroll
            for (int i = 0; i < kMaxTimes; ++i)
              if (i < nt) dump_val[o + i] = Pt[i];
            if (dump_segs != nullptr) dump_segs[(int64_t)point * trees + (int64_t)tree] = segs;
          }
        }
        // finished trees enter the wave's sums in lane order: the tree's lane
        // stages its values in LDS, lane i adds value i to time i's sums
        uint64_t dmask = ballot(done);
        const uint64_t dmask0 = dmask;
        double* const row = &wrow[wid][0];
        while (dmask != 0) {
          const int l = __builtin_ctzll(dmask);
          dmask &= dmask - 1;
          __builtin_amdgcn_wave_barrier();
          if (lane == l) {
#pragma unroll
            for (int i = 0; i < kMaxTimes; ++i) row[i] = Pt[i];
          }
          __builtin_amdgcn_wave_barrier();
          if (lane < nt) {
            const double v = row[lane];
            const bool first = W[3 * kMaxTimes] == 0.0;
            const double K = first ? v : W[2 * kMaxTimes + lane];
            if (first) W[2 * kMaxTimes + lane] = v;
            const double dv = v - K;
            W[lane] += dv;
            W[kMaxTimes + lane] += dv * dv;
          }
          __builtin_amdgcn_wave_barrier();
          if (lane == 0) W[3 * kMaxTimes] += 1.0;
          __builtin_amdgcn_wave_barrier();
        }
        // refill
        if (dmask0 != 0) {
          const uint32_t ntr = cursor + (uint32_t)lane_rank(dmask0);
          cursor += (uint32_t)__popcll(dmask0);
          if (done) {
            if (ntr < pend) {
              tree = ntr;
              attempt = 0;
              start_tree();
            } else {
              active = false;
            }
          }
        }
        ev = 0;
      }
    }

    lsub = wave_sum(lsub);
    lcens = wave_sum(lcens);
    lredraw = wave_sum(lredraw);
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) {
      const double n = W[3 * kMaxTimes];
      for (int i = 0; i < nt; ++i) {
        ItemStat st;
        const double a = n > 0.0 ? W[i] / n : 0.0;
        st.mean = n > 0.0 ? W[2 * kMaxTimes + i] + a : 0.0;
        const double m2 = W[kMaxTimes + i] - W[i] * a;
        st.m2 = m2 > 0.0 ? m2 : 0.0;
        st.n = (int64_t)n;
        st.steps = lsub;
        st.censored = lcens;
        st.redrawn = i == 0 ? lredraw : 0;
        istat[(int64_t)i * n_items + it.slot] = st;
      }
    }
  }
}

}  // namespace pdd
