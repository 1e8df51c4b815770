// Heterogeneous batch of linear problems in one persistent launch (the loops
// over interface nodes and their samples of Algorithm 3.1, across subdomains
// whose domains and data differ, as in a PDD partition): every work item
// (node, path range) carries its node, the node carries its problem, and the
// problem's record (domain, sigma sqrt(dt), the polynomials of b, c, f, the
// data g) is read through scalar loads when a wavefront takes the item.  One
// queue holds all items, large ones first and longest first within a size
// class, so problems of different dimension and cost share one grid.
//
// The per-item walk is the forward k_walk's (Euler-Maruyama with the exit
// test, or walk on spheres; FP32 or FP64 stepping, FP64 Welford per item)
// with the same arithmetic in the same order, so a path's value equals the
// single-problem kernel's and the oracle's on the same counters.  b, c, f
// are dense polynomials (of degree <= 3) here, g may have generic terms.
#include <hip/hip_runtime.h>

#include "pdd_device.hpp"
#include "pdd_kernels.hpp"
#include "walk_kernels.hpp"

namespace pdd {

template <typename R>
__device__ __forceinline__ Dom<R> batch_dom(const LinearParams PDD_CONST_AS* P, bool test);
template <>
__device__ __forceinline__ Dom<float> batch_dom<float>(const LinearParams PDD_CONST_AS* P, bool test) {
  Dom<float> D;
  D.kind = P->dom_kind;
  for (int k = 0; k < 3; ++k) {
    D.lo[k] = test ? P->tlof[k] : P->lof[k];
    D.hi[k] = test ? P->thif[k] : P->hif[k];
    D.ctr[k] = P->ctrf[k];
  }
  D.rad = P->radf;
  D.rad2 = test ? P->trad2f : P->rad2f;
  return D;
}
template <>
__device__ __forceinline__ Dom<double> batch_dom<double>(const LinearParams PDD_CONST_AS* P, bool test) {
  Dom<double> D;
  D.kind = P->dom_kind;
  for (int k = 0; k < 3; ++k) {
    D.lo[k] = test ? P->tlo[k] : P->lo[k];
    D.hi[k] = test ? P->thi[k] : P->hi[k];
    D.ctr[k] = P->ctr[k];
  }
  D.rad = P->rad;
  D.rad2 = test ? P->trad2 : P->rad2;
  return D;
}

template <typename R>
__device__ __forceinline__ R batch_dt(const LinearParams PDD_CONST_AS* P) {
  if constexpr (sizeof(R) == 4) return P->dtf; else return P->dt;
}
template <typename R>
__device__ __forceinline__ R batch_sdt(const LinearParams PDD_CONST_AS* P) {
  if constexpr (sizeof(R) == 4) return P->sdtf; else return P->sdt;
}

// The staged coefficient table as scalar loads (float or double copy).
template <typename R>
__device__ __forceinline__ const R PDD_CONST_AS* batch_coefs(const double* cd, const float* cf) {
  if constexpr (sizeof(R) == 4) return (const R PDD_CONST_AS*)const_table(cf);
  else return (const R PDD_CONST_AS*)const_table(cd);
}

// The exit test of a problem whose domain kind is KIND, with the bounds (box)
// or the centre and squared radius (ball) held in vector registers in FP32,
// so the comparisons that read them can share an issue slot; the same
// arithmetic as inside().
template <typename R, int DIM, int KIND>
struct ExitTest {
  R lo[DIM], hi[DIM], ctr[DIM], rad2;
  __device__ __forceinline__ explicit ExitTest(const Dom<R>& D) {
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      lo[k] = D.lo[k];
      hi[k] = D.hi[k];
      ctr[k] = D.ctr[k];
    }
    rad2 = D.rad2;
    if constexpr (sizeof(R) == 4) {
#pragma unroll
      for (int k = 0; k < DIM; ++k) {
        if constexpr (KIND == DOM_BOX) asm volatile("" : "+v"(lo[k]), "+v"(hi[k]));
        else asm volatile("" : "+v"(ctr[k]));
      }
      if constexpr (KIND != DOM_BOX) asm volatile("" : "+v"(rad2));
    }
  }
  __device__ __forceinline__ bool inside(const R* x) const {
    if constexpr (KIND == DOM_BOX) {
      bool in = true;
#pragma unroll
      for (int k = 0; k < DIM; ++k) in = in && (x[k] > lo[k]) && (x[k] < hi[k]);
      return in;
    } else {
      R r2 = (R)0;
#pragma unroll
      for (int k = 0; k < DIM; ++k) {
        const R d = x[k] - ctr[k];
        r2 += d * d;
      }
      return r2 < rad2;
    }
  }
};

// The paths [it.p0, it.p0 + it.count) of one node of a DIM-dimensional
// problem whose domain kind is KIND: stepping, parking ended paths as exit
// records, refilling lanes, flushing records 64 at a time, and the item's
// statistics into istat.  BCF = false is the instance for problems with
// b = c = f = 0 (pure diffusion): the step has no drift, killing or source
// code and no per-step tests of the problem's flags, which otherwise cost a
// scalar branch each (C3, all Laplacian: 36.4 -> 30.9 ms).
template <typename R, int DIM, int LAYOUT, bool WOS, int KIND, bool BCF>
__device__ __forceinline__ void batch_item(const LinearParams PDD_CONST_AS* P, const WorkItem it,
                                           const double* __restrict__ nodes, const DevFactor* __restrict__ fac,
                                           const double* __restrict__ cd, const float* __restrict__ cf, uint32_t k0,
                                           uint32_t k1, int refill_groups, R* rec, uint32_t* rec_path,
                                           uint32_t* rec_n, int lane, ItemStat* __restrict__ istat,
                                           double* __restrict__ dump_phi, int64_t* __restrict__ dump_steps,
                                           const int64_t* __restrict__ dump_off) {
  using NZr = Normals<R, LAYOUT>;
  using GS = GroupShape<DIM, NZr::kPerBlock>;
  constexpr int NM = GradedLex<DIM, kMaxPolyBCF>::N;
  const Dom<R> D = batch_dom<R>(P, false);
  const Dom<R> Dt = batch_dom<R>(P, true);
  const ExitTest<R, DIM, KIND> exit_test(Dt);
  R dt = batch_dt<R>(P);
  R sdt = batch_sdt<R>(P);
  if constexpr (sizeof(R) == 4) asm volatile("" : "+v"(dt), "+v"(sdt));
  const uint32_t max_steps = (uint32_t)P->max_steps;
  const bool has_b = BCF && P->has_b != 0, has_c = BCF && P->has_c != 0, has_f = BCF && P->has_f != 0;
  const bool need_mono = has_b || has_c || has_f;
  const int node = it.node;
  const uint32_t pend = it.p0 + it.count;

  R x0[DIM];
#pragma unroll
  for (int k = 0; k < DIM; ++k) x0[k] = to_r<R>(nodes[(size_t)node * 3 + k]);
  const bool node_in = inside<R, DIM>(Dt, x0);

  uint32_t path = it.p0 + (uint32_t)lane;
  bool alive = (path < pend) && node_in;
  bool fin = (path < pend) && !node_in;
  bool cens = false;
  uint32_t cursor = it.p0 + (it.count < (uint32_t)kWave ? it.count : (uint32_t)kWave);
  R X[DIM];
#pragma unroll
  for (int k = 0; k < DIM; ++k) X[k] = x0[k];
  R Y = (R)1, Z = (R)0;
  uint32_t n = 0;
  double wn = 0.0, wmean = 0.0, wm2 = 0.0;
  int64_t lsteps = 0, lcens = 0;
  int nrec = 0;

  auto flush = [&]() {
    if (nrec == 0) return;
    __builtin_amdgcn_wave_barrier();
    if (lane < nrec) {
      R xe[DIM];
#pragma unroll
      for (int k = 0; k < DIM; ++k) xe[k] = rec[k * kWave + lane];
      const R y = rec[DIM * kWave + lane], z = rec[(DIM + 1) * kWave + lane];
      const uint32_t pr = rec_path[lane], nr = rec_n[lane];
      R xr[3];
      project<R, DIM>(D, xe, xr);
      DevFun g;
      g.n_terms = P->g.n_terms;
      g.n_factors = P->g.n_factors;
      g.fac_off = P->g.fac_off;
      g.coef_off = P->g.coef_off;
      g.poly_deg = P->g.poly_deg;
      g.n_mono = P->g.n_mono;
      g.poly_off = P->g.poly_off;
      g.pad = 0;
      R gv = (R)0;
      if (g.n_terms > 0) gv = terms_sum<R, DIM>(fac, cd, cf, g, xr);
      if (g.poly_deg >= 0) gv += poly_nested<R, DIM>(cd, cf, g.poly_deg, g.poly_off, xr);
      const R phi = gv * y + z;
      const double ph = (double)phi;
      wn += 1.0;
      const double d1 = ph - wmean;
      wmean += d1 / wn;
      wm2 += d1 * (ph - wmean);
      lsteps += (int64_t)(nr & 0x7FFFFFFFu);
      lcens += (int64_t)(nr >> 31);
      if (dump_phi != nullptr) {
        const int64_t o = dump_off[node] + (int64_t)pr;
        dump_phi[o] = ph;
        if (dump_steps != nullptr) dump_steps[o] = (int64_t)(nr & 0x7FFFFFFFu);
      }
    }
    __builtin_amdgcn_wave_barrier();
    nrec = 0;
  };

  for (;;) {
    for (int gi = 0; gi < refill_groups; ++gi) {
      if (!__any(alive)) break;
      R z[GS::NZ];
      {
        const uint64_t blk0 = ((uint64_t)n * DIM) / NZr::kPerBlock;
#pragma unroll
        for (int b = 0; b < GS::NB; ++b) {
          const uint64_t blk = blk0 + (uint64_t)b;
          uint32_t ka = k0, kb = k1;
          asm volatile("" : "+s"(ka), "+s"(kb));
          NZr::gen((uint32_t)blk, (uint32_t)((blk >> 32) & 0xFFFFFFu), path, (uint32_t)node, ka, kb,
                   &z[b * NZr::kPerBlock]);
        }
      }
#pragma unroll
      for (int s = 0; s < GS::G; ++s) {
        if constexpr (WOS) {
          // predicated like the pure-diffusion Euler step below: a lane that
          // stops or is inactive jumps by a radius of 0, an active one by the
          // same operations as a branched jump (C3: 4.38 -> 4.07 ms)
          const bool act = alive && n < max_steps;
          const R r = boundary_distance<R, DIM>(D, X);
          const bool stop = act && !(r >= dt);
          const bool jump = act && (r >= dt);
          const R z2 = sum_squares<R, DIM>(&z[s * DIM]);
          jump_sphere<R, DIM>(X, jump ? r : (R)0, z2, &z[s * DIM]);
          n += jump ? 1u : 0u;
          alive = alive && !stop;
          fin = fin || stop;
          continue;
        }
        if constexpr (!BCF) {
          // pure diffusion, predicated instead of branched: the per-step
          // branch's exec-mask bookkeeping is scalar work, and the scalar
          // unit bounds this kernel (C3: 30.8 -> 27.5 ms).  An inactive lane
          // adds 0 z; an active one takes the same fused multiply-add as the
          // branched step, so paths and exit steps are unchanged.
          const bool act = alive && n < max_steps;
          const R m = act ? sdt : (R)0;
#pragma unroll
          for (int k = 0; k < DIM; ++k) X[k] = X[k] + m * z[s * DIM + k];
          n += act ? 1u : 0u;
          const bool out = act && !exit_test.inside(X);
          alive = alive && !out;
          fin = fin || out;
          continue;
        }
        if (alive && n < max_steps) {
          R mono[NM];
          if (need_mono) monomials<R, DIM, kMaxPolyBCF>(X, mono);
          const R PDD_CONST_AS* ct = batch_coefs<R>(cd, cf);
          if (has_f) Z = Z + poly_dot<R, NM>(ct + P->f.poly_off, mono) * Y * dt;
          if (has_c) Y = Y * fexp(-poly_dot<R, NM>(ct + P->c.poly_off, mono) * dt);
          if (has_b) {
            R bv[DIM];
#pragma unroll
            for (int k = 0; k < DIM; ++k)
              bv[k] = P->b[k].poly_deg >= 0 ? poly_dot<R, NM>(ct + P->b[k].poly_off, mono) : (R)0;
#pragma unroll
            for (int k = 0; k < DIM; ++k) X[k] = X[k] + bv[k] * dt + sdt * z[s * DIM + k];
          } else {
#pragma unroll
            for (int k = 0; k < DIM; ++k) X[k] = X[k] + sdt * z[s * DIM + k];
          }
          ++n;
          if (!exit_test.inside(X)) {
            alive = false;
            fin = true;
          }
        }
      }
    }
    if (alive && n >= max_steps) {
      alive = false;
      fin = true;
      cens = WOS ? (boundary_distance<R, DIM>(D, X) >= dt) : true;
    }

    // park ended paths in LDS, refill their lanes with the item's next paths
    const uint64_t fmask = ballot(fin);
    if (fmask != 0) {
      const int nf = __popcll(fmask);
      if (nrec + nf > kWave) flush();
      if (fin) {
        const int slot = nrec + lane_rank(fmask);
#pragma unroll
        for (int k = 0; k < DIM; ++k) rec[k * kWave + slot] = X[k];
        rec[DIM * kWave + slot] = Y;
        rec[(DIM + 1) * kWave + slot] = Z;
        rec_path[slot] = path;
        rec_n[slot] = n | (cens ? 0x80000000u : 0u);
      }
      nrec += nf;
      const uint32_t np = cursor + (uint32_t)lane_rank(fmask);
      cursor += (uint32_t)nf;
      if (fin) {
        fin = false;
        cens = false;
        if (np < pend) {
          path = np;
#pragma unroll
          for (int k = 0; k < DIM; ++k) X[k] = x0[k];
          Y = (R)1;
          Z = (R)0;
          n = 0;
          alive = node_in;
          fin = !node_in;
        } else {
          path = pend;
        }
      }
    }
    if (!__any(alive) && !__any(fin)) break;
  }

  flush();
  wave_welford(wn, wmean, wm2);
  lsteps = wave_sum(lsteps);
  lcens = wave_sum(lcens);
  if (lane == 0) {
    ItemStat st;
    st.mean = wmean;
    st.m2 = wm2;
    st.n = (int64_t)wn;
    st.steps = lsteps;
    st.censored = lcens;
    st.redrawn = 0;
    istat[it.slot] = st;
  }
}

// FP32: built for six waves per SIMD (at most 80 VGPRs), so the default six
// blocks per CU are all resident: the Euler instance needed 81 VGPRs for
// five waves; at 79 with six it is 1-2% faster on C3, without scratch.
template <typename R, int LAYOUT, bool WOS>
__global__ void __launch_bounds__(kBlock, (sizeof(R) == 4 ? 6 : 1))
k_walk_batch(const LinearParams* __restrict__ probs, const int32_t* __restrict__ node_prob,
             const double* __restrict__ nodes, const DevFactor* __restrict__ fac, const double* __restrict__ cd,
             const float* __restrict__ cf, uint32_t k0, uint32_t k1, const WorkItem* __restrict__ items, int n_items,
             uint32_t* __restrict__ qhead, ItemStat* __restrict__ istat, double* __restrict__ dump_phi,
             int64_t* __restrict__ dump_steps, const int64_t* __restrict__ dump_off, int refill_groups) {
  constexpr int kWaves = kBlock / kWave;
  __shared__ R area[kWaves][5 * kWave];        // exit records: X (up to 3), Y, Z, field-major
  __shared__ uint32_t rec_i[kWaves][2][kWave];  // path, steps | censored << 31
  const int lane = (int)(threadIdx.x & (kWave - 1));
  const int wid = (int)(threadIdx.x / kWave);
  for (;;) {
    const uint32_t it_idx = pop_item(qhead);
    if (it_idx >= (uint32_t)n_items) break;
    const WorkItem it = items[it_idx];
    const int k = __builtin_amdgcn_readfirstlane(node_prob[it.node]);
    const LinearParams PDD_CONST_AS* P = const_table(probs) + k;
    const bool box = P->dom_kind == DOM_BOX;
    // walk on spheres requires b = c = f = 0
    const bool bcf = !WOS && (P->has_b != 0 || P->has_c != 0 || P->has_f != 0);
#define PDD_BATCH_ITEM_B(DIM, KIND, BCF)                                                                         \
  batch_item<R, DIM, LAYOUT, WOS, KIND, BCF>(P, it, nodes, fac, cd, cf, k0, k1, refill_groups, area[wid],          \
                                             rec_i[wid][0], rec_i[wid][1], lane, istat, dump_phi, dump_steps, dump_off)
#define PDD_BATCH_ITEM(DIM, KIND)                 \
  do {                                            \
    if (bcf) PDD_BATCH_ITEM_B(DIM, KIND, true);   \
    else PDD_BATCH_ITEM_B(DIM, KIND, false);      \
  } while (0)
    switch (P->dim) {
      case 1:
        if (box) PDD_BATCH_ITEM(1, DOM_BOX);
        else PDD_BATCH_ITEM(1, DOM_BALL);
        break;
      case 2:
        if (box) PDD_BATCH_ITEM(2, DOM_BOX);
        else PDD_BATCH_ITEM(2, DOM_BALL);
        break;
      default:
        if (box) PDD_BATCH_ITEM(3, DOM_BOX);
        else PDD_BATCH_ITEM(3, DOM_BALL);
        break;
    }
#undef PDD_BATCH_ITEM
#undef PDD_BATCH_ITEM_B
  }
}

template <typename R, int LAYOUT, bool WOS>
static hipError_t launch_batch_t(const WalkBatchLaunch& L, hipStream_t st) {
  hipLaunchKernelGGL((k_walk_batch<R, LAYOUT, WOS>), dim3(L.grid), dim3(kBlock), 0, st, L.probs, L.node_prob, L.nodes,
                     L.fac, L.cd, L.cf, L.key0, L.key1, L.items, L.n_items, L.qhead, L.istat, L.dump_phi,
                     L.dump_steps, L.dump_off, L.refill_groups);
  return hipGetLastError();
}

hipError_t launch_walk_batch(const WalkBatchLaunch& L, hipStream_t st) {
  if (L.fp32) return L.wos ? launch_batch_t<float, RNG_QUAD24, true>(L, st) : launch_batch_t<float, RNG_QUAD24, false>(L, st);
  if (L.layout == RNG_QUAD24)
    return L.wos ? launch_batch_t<double, RNG_QUAD24, true>(L, st) : launch_batch_t<double, RNG_QUAD24, false>(L, st);
  return L.wos ? launch_batch_t<double, RNG_PAIR52, true>(L, st) : launch_batch_t<double, RNG_PAIR52, false>(L, st);
}

}  // namespace pdd
