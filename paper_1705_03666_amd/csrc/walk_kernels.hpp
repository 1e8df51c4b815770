// Feynman-Kac walk kernels (Sec. 2.2, eqs. 2.7-2.9 in the elliptic
// pure-Dirichlet limit; Euler-Maruyama plus boundary test, Sec. 2.1).
//
//  k_walk<R, DIM, DFC, LAYOUT, TERMS, ADJ>  persistent batched kernel: every
//      wavefront pops work items (node, path range) from a device queue and
//      runs one path per lane; a lane whose path has exited takes the next
//      path index of the item ("refill"), so lanes stay busy while exit times
//      vary tenfold.  R = float: FP32 stepping / transforms; R = double: FP64.
//      DFC = 3: b, c, f carry a dense cubic part; TERMS: they (or g, for the
//      adjoint) carry generic terms.  With ADJ the same paths are simulated
//      with pathwise tangents and the derivative of each path value with
//      respect to the coefficients of g, f and c is accumulated per item (the
//      exact derivative of the discrete estimator).
//  k_walk_plain<DIM, DFC, LAYOUT>  the FP64 baseline: one node per launch,
//      one path per thread until it exits, block-level partial statistics.
//
// Path p of node i draws its Gaussians from Philox counters
// (block, stream 0 | block >> 32, p, i): the path is a pure function of
// (seed, i, p), independent of which lane or launch computes it.
#pragma once
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#endif

#include "pdd_device.hpp"
#ifndef __HIPCC_RTC__
#include "pdd_kernels.hpp"
#endif

namespace pdd {

constexpr int gcd_c(int a, int b) { return b == 0 ? a : gcd_c(b, a % b); }

// G consecutive steps consume NZ = G*DIM Gaussians = NB whole Philox blocks.
template <int DIM, int PB>
struct GroupShape {
  static constexpr int L = DIM * PB / gcd_c(DIM, PB);
  static constexpr int G = L / DIM;
  static constexpr int NZ = L;
  static constexpr int NB = L / PB;
};

template <typename R>
__device__ __forceinline__ R to_r(double v) { return (R)v; }

// b, c, f at X (terms + dense polynomial).  The monomials are computed once
// and shared by every function that has a polynomial part.
template <typename R, int DIM, int DFC>
struct BCF {
  static constexpr int NM = GradedLex<DIM, DFC>::N;
  R mono[NM > 0 ? NM : 1];
  R b[DIM];
  R c, f;
};

template <typename R, int DIM, int DFC>
__device__ __forceinline__ R poly_graded(const LinearParams& P, const DevFun& F, const R* mono) {
  constexpr int NM = GradedLex<DIM, DFC>::N;
  R s = (R)0;
#pragma unroll
  for (int m = 0; m < NM; ++m) s += coef_at<R>(P.cd, P.cf, F.poly_off + m) * mono[m];
  return s;
}

template <typename R, int DIM, int DFC>
__device__ __forceinline__ R fun_value(const LinearParams& P, const DevFun& F, const R* X, const R* mono) {
  R v = (R)0;
  if (F.n_terms > 0) v = terms_sum<R, DIM>(P.fac, P.cd, P.cf, F, X);
  if constexpr (DFC >= 0) {
    if (F.poly_deg >= 0) v += poly_graded<R, DIM, DFC>(P, F, mono);
  }
  return v;
}

template <typename R, int DIM>
__device__ __forceinline__ R g_value(const LinearParams& P, const R* xp) {
  R v = (R)0;
  if (P.g.n_terms > 0) v = terms_sum<R, DIM>(P.fac, P.cd, P.cf, P.g, xp);
  if (P.g.poly_deg >= 0) v += poly_nested<R, DIM>(P.cd, P.cf, P.g.poly_deg, P.g.poly_off, xp);
  return v;
}

template <typename R>
__device__ __forceinline__ R dt_of(const LinearParams& P);
template <>
__device__ __forceinline__ float dt_of<float>(const LinearParams& P) { return P.dtf; }
template <>
__device__ __forceinline__ double dt_of<double>(const LinearParams& P) { return P.dt; }
template <typename R>
__device__ __forceinline__ R sdt_of(const LinearParams& P);
template <>
__device__ __forceinline__ float sdt_of<float>(const LinearParams& P) { return P.sdtf; }
template <>
__device__ __forceinline__ double sdt_of<double>(const LinearParams& P) { return P.sdt; }

// Coefficient tables of the dense polynomials, read as scalar loads (see
// const_table).
template <typename R>
__device__ __forceinline__ const R PDD_CONST_AS* coef_table(const LinearParams& P);
template <>
__device__ __forceinline__ const float PDD_CONST_AS* coef_table<float>(const LinearParams& P) {
  uint64_t a = reinterpret_cast<uint64_t>(P.cf);
  asm volatile("" : "+s"(a));
  return (const float PDD_CONST_AS*)a;
}
template <>
__device__ __forceinline__ const double PDD_CONST_AS* coef_table<double>(const LinearParams& P) {
  uint64_t a = reinterpret_cast<uint64_t>(P.cd);
  asm volatile("" : "+s"(a));
  return (const double PDD_CONST_AS*)a;
}

// Dense graded-lex polynomial: c[0] + sum_m c[m] mono[m] (mono[0] = 1).
template <typename R, int NM>
__device__ __forceinline__ R poly_dot(const R PDD_CONST_AS* c, const R* mono) {
  R s = c[0];
#pragma unroll
  for (int m = 1; m < NM; ++m) s += c[m] * mono[m];
  return s;
}

// The same with the coefficients in LDS: every lane reads the same address
// (a broadcast, four coefficients per read), and the products then take
// only VGPR operands, so they can share an issue slot with another
// wavefront's instruction that reads a scalar register.
template <typename R, int NM>
__device__ __forceinline__ R poly_dot_lds(const __attribute__((address_space(3))) R* c, const R* mono) {
  R s = c[0];
#pragma unroll
  for (int m = 1; m < NM; ++m) s += c[m] * mono[m];
  return s;
}

// The six coefficient functions of a linear problem, as template arguments.
enum : int { FUN_B0 = 0, FUN_B1 = 1, FUN_B2 = 2, FUN_C = 3, FUN_F = 4, FUN_G = 5 };

template <int W>
__device__ __forceinline__ const DevFun& fun_of(const LinearParams& P) {
  if constexpr (W <= FUN_B2) return P.b[W];
  else if constexpr (W == FUN_C) return P.c;
  else if constexpr (W == FUN_F) return P.f;
  else return P.g;
}

// Generic-term evaluation policies of k_walk.  TableTerms interprets the
// staged factor records at run time (any problem).  A problem-specialised
// policy, generated as source and compiled at run time, has the same members
// with the factor structure (functions, coordinates, scales, shifts, powers)
// written in as constants; it evaluates the same products in the same order.
//   State<R>                  per-thread data loaded once per launch
//   load<R>(P)                builds it (the specialised policy copies the
//                             term coefficients of b, c and f into VGPRs, so
//                             the per-step products read no scalar register)
//   sum<R, DIM, W>(P, st, x)  sum over the terms t of function W of coef_t term_t(x)
//   term<R, DIM, W>(P, t, x)  term_t(x) without its coefficient
struct TableTerms {
  template <typename R>
  struct State {};
  template <typename R>
  __device__ static __forceinline__ State<R> load(const LinearParams&) {
    return State<R>{};
  }
  template <typename R, int DIM, int W>
  __device__ static __forceinline__ R sum(const LinearParams& P, const State<R>&, const R* x) {
    return terms_sum<R, DIM>(P.fac, P.cd, P.cf, fun_of<W>(P), x);
  }
  template <typename R, int DIM, int W>
  __device__ static __forceinline__ R term(const LinearParams& P, int t, const R* x) {
    return term_value<R, DIM>(P.fac, fun_of<W>(P), t, x);
  }
};

// b_k, c or f at X: generic terms (only when TERMS) plus the dense polynomial.
template <typename R, int DIM, int DFC, bool TERMS, class TP, int W>
__device__ __forceinline__ R bcf_value(const LinearParams& P, const typename TP::template State<R>& st,
                                       const DevFun& F, const R* X, const R* mono) {
  R v = (R)0;
  if constexpr (TERMS) {
    if (F.n_terms > 0) v = TP::template sum<R, DIM, W>(P, st, X);
  }
  if constexpr (DFC >= 0) {
    if (F.poly_deg >= 0) v += poly_dot<R, GradedLex<DIM, DFC>::N>(coef_table<R>(P) + F.poly_off, mono);
  }
  return v;
}

// g at the projected exit point: generic terms plus the nested polynomial.
template <typename R, int DIM, class TP>
__device__ __forceinline__ R g_value_tp(const LinearParams& P, const typename TP::template State<R>& st,
                                        const R* xp) {
  R v = (R)0;
  if (P.g.n_terms > 0) v = TP::template sum<R, DIM, FUN_G>(P, st, xp);
  if (P.g.poly_deg >= 0) v += poly_nested<R, DIM>(P.cd, P.cf, P.g.poly_deg, P.g.poly_off, xp);
  return v;
}

// Persistent batched walk.  Every wavefront pops work items (node, path range)
// from a device queue and runs one path per lane; a lane whose path has ended
// takes the next path index of the item, so lanes stay busy while exit times
// vary tenfold.  Ended paths are parked in LDS as exit records (X, Y, Z and,
// for the adjoint, the tangent S) and processed 64 at a time, one record per
// lane: projection onto the boundary, g, the path value phi = g Y + Z, the
// FP64 Welford update and the g-part of the derivative.
//
// Adjoint (ADJ).  With Z_{n+1} = Z_n + f(X_n) Y_n dt, Y_{n+1} = Y_n
// exp(-c(X_n) dt) and phi = g(X_N) Y_N + Z_N, the exact derivatives of the
// discrete path value with respect to a coefficient theta_j of f (basis
// function m_j) and of c are
//   d phi / d f_j = F_j = sum_n m_j(X_n) Y_n dt,
//   d phi / d c_j = -phi S_j + B_j,  S_j = sum_n m_j(X_n) dt,
//                                    B_j = sum_n m_j(X_n) dt Z_{n+1},
// (summation by parts of -g Y_N S_j(N) - sum_n f_n Y_n dt S_j(n)).  F and B
// need no per-path reset, so each lane keeps them as running sums over all
// the paths it runs; only S is per path and travels with the exit record.
// The lanes sum F/dt, S/dt and B/dt (dt is the same at every step), and the
// factor dt is applied once, when the running sums are folded: the stepping
// loop then adds m_j, m_j Y and m_j Z with no scalar-register operand, so
// those updates can issue in the same cycle as another wavefront's
// instruction that reads one.
// At every record flush the running sums are reduced across the wavefront
// into FP64 per-item accumulators (column ic lives in lane ic % 64, slot
// ic / 64), so no FP32 sum spans more than about one path per lane.
// Occupancy request: the FP32 kernels without generic terms fit in 128 VGPRs
// (four waves per SIMD), those with terms in 256; the FP64 kernels (parity
// and baseline use) are left unconstrained.
template <typename R, bool TERMS>
constexpr int walk_min_waves() { return sizeof(R) == 4 ? (TERMS ? 2 : 4) : 1; }

template <typename R, int DIM, int DFC, int LAYOUT, bool TERMS, bool ADJ, bool WOS = false, class TP = TableTerms>
__global__ void __launch_bounds__(kBlock, (walk_min_waves<R, TERMS>()))
k_walk(const LinearParams P, const WorkItem* __restrict__ items, int n_items, uint32_t* __restrict__ qhead,
       ItemStat* __restrict__ istat, double* __restrict__ igrad, int grad_stride,
       double* __restrict__ dump_phi, int64_t* __restrict__ dump_steps, const int64_t* __restrict__ dump_off,
       int refill_groups) {
  using NZr = Normals<R, LAYOUT>;
  using GS = GroupShape<DIM, NZr::kPerBlock>;
  constexpr int NM = GradedLex<DIM, DFC>::N;
  constexpr int NT = (ADJ && TERMS) ? kAdjTerms : 0;
  constexpr int NP = ADJ ? NT + NM : 0;
  constexpr int kRecW = DIM + 2 + NP;
  constexpr int kWaves = kBlock / kWave;
  constexpr int kGMono = GradedLex<DIM, kMaxPolyG>::N;      // g-polynomial monomials, at most
  constexpr int kCols = ADJ ? 2 * NP + NT + kGMono : 0;
  constexpr int kSlots = kCols > 0 ? (kCols + kWave - 1) / kWave : 1;
  constexpr int kGSlots = (kGMono + kWave - 1) / kWave;
  // power table of the g-gradient pass, one row of odd stride per record:
  // Y x0^a (a = 0..deg), x1^b, x2^c (b, c = 1..deg), and a constant 1
  constexpr int kPwStride = (DIM * kMaxPolyG + 2) | 1;
  constexpr int kFoldMax = NP > NT ? NP : (NT > 0 ? NT : 1);
  constexpr int kArea0 = kRecW * kWave;
  constexpr int kArea1 = ADJ ? kWave * kPwStride : 0;
  constexpr int kArea2 = ADJ ? kWave * (kFoldMax | 1) : 0;
  constexpr int kArea = kArea0 > kArea1 ? (kArea0 > kArea2 ? kArea0 : kArea2) : (kArea1 > kArea2 ? kArea1 : kArea2);

  const int lane = (int)(threadIdx.x & (kWave - 1));
  const int wid = (int)(threadIdx.x / kWave);
  // Per-wave scratch, used in turn as (1) the exit records, field-major with
  // one column per record (conflict-free lane-per-record reads), (2) the
  // power table of the g-gradient pass and (3) the transpose of the
  // running derivative sums.
  __shared__ R area[kWaves][kArea];
  __shared__ uint32_t rec_i[kWaves][2][kWave];   // path, steps | censored << 31
  // FP64 per-item derivative accumulators, column ic at [ic / 64][ic % 64]
  __shared__ double acc[ADJ ? kWaves : 1][kSlots][kWave];
  // g-polynomial monomial k (nested order): its three power-table rows
  __shared__ uint32_t gmono[ADJ ? kGMono : 1];
  // The adjoint keeps the statistics of the current item per wavefront in
  // LDS (FP64 Welford triple (n, mean, M2), step and censoring counts),
  // merged at every flush, so no lane holds FP64 or 64-bit accumulators
  // through its register-bound stepping loop; the forward kernels, whose
  // steps are short, keep them per lane (cheaper flushes).
  constexpr bool kWaveStats = ADJ;
  __shared__ double wstat[kWaveStats ? kWaves : 1][3];
  __shared__ int64_t wcount[kWaveStats ? kWaves : 1][2];
  R* const rec = &area[wid][0];
  // FP32 walks without generic terms: the dense coefficients of c and f are
  // copied into LDS once per block and read from there at every step (the
  // table-read form makes 40 of the step's FMAs read SGPRs)
  constexpr bool kLdsPoly = sizeof(R) == 4 && !TERMS && !WOS && DFC >= 0;
  constexpr int kNMc = GradedLex<DIM, (DFC >= 0 ? DFC : 0)>::N;
  constexpr int kNMp = ((kNMc + 3) / 4) * 4;      // 16-byte aligned rows
  __shared__ __attribute__((aligned(16))) R lpoly[kLdsPoly ? 2 * kNMp : 4];   // row 0: c, row 1: f
  if constexpr (kLdsPoly) {
    for (int i = (int)threadIdx.x; i < 2 * kNMp; i += kBlock) {
      const DevFun& F = i < kNMp ? P.c : P.f;
      const int m = i % kNMp;
      lpoly[i] = (F.poly_deg >= 0 && m < kNMc) ? P.cf[F.poly_off + m] : (R)0;
    }
    __syncthreads();
  }

  const Dom<R> D = make_dom<R>(P);          // projection of exit points
  const Dom<R> Dt = make_test_dom<R>(P);    // exit test
  R dt = dt_of<R>(P);
  R sdt = sdt_of<R>(P);
  // FP32: keep the step sizes in VGPRs, so the products that use them read no
  // SGPR and can share an issue slot with another wavefront's instruction
  if constexpr (sizeof(R) == 4) asm volatile("" : "+v"(dt), "+v"(sdt));
  const typename TP::template State<R> tst = TP::template load<R>(P);
  const uint32_t max_steps = (uint32_t)P.max_steps;
  const uint32_t k0 = P.key0, k1 = P.key1;
  const int ngm = (ADJ && P.g.poly_deg >= 0) ? P.g.n_mono : 0;
  if constexpr (ADJ) {
    if (P.g.poly_deg >= 0 && threadIdx.x == 0) {
      const int deg = P.g.poly_deg, one = DIM * deg + 1;
      int k = 0;
      for (int ea = 0; ea <= deg; ++ea)
        for (int eb = 0; eb <= (DIM >= 2 ? deg - ea : 0); ++eb)
          for (int ec = 0; ec <= (DIM >= 3 ? deg - ea - eb : 0); ++ec) {
            const uint32_t rb = eb > 0 ? (uint32_t)(deg + eb) : (uint32_t)one;
            const uint32_t rc = ec > 0 ? (uint32_t)(2 * deg + ec) : (uint32_t)one;
            gmono[k++] = (uint32_t)ea | (rb << 8) | (rc << 16);
          }
    }
    __syncthreads();
  }

  for (;;) {
    const uint32_t it_idx = pop_item(qhead);
    if (it_idx >= (uint32_t)n_items) break;
    const WorkItem it = items[it_idx];
    const int node = it.node;
    const uint32_t pend = it.p0 + it.count;

    R x0[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) x0[k] = to_r<R>(P.nodes[(size_t)node * DIM + k]);
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

    double wn = 0.0, wmean = 0.0, wm2 = 0.0;   // per lane (forward kernels)
    int64_t lsteps = 0, lcens = 0;
    if constexpr (kWaveStats) {
      if (lane == 0) {
        wstat[wid][0] = 0.0;
        wstat[wid][1] = 0.0;
        wstat[wid][2] = 0.0;
        wcount[wid][0] = 0;
        wcount[wid][1] = 0;
      }
    }
    int nrec = 0;

    R S[NP > 0 ? NP : 1], Fr[NP > 0 ? NP : 1], Br[NP > 0 ? NP : 1], Gr[NT > 0 ? NT : 1];
#pragma unroll
    for (int j = 0; j < NP; ++j) S[j] = Fr[j] = Br[j] = (R)0;
#pragma unroll
    for (int t = 0; t < NT; ++t) Gr[t] = (R)0;
    if constexpr (ADJ) {
#pragma unroll
      for (int r = 0; r < kSlots; ++r) acc[wid][r][lane] = 0.0;
    }

    // Folds CNT running sums v[] of every lane into accumulator columns
    // ic0.. through an LDS transpose: lane j then adds up column j in FP64.
    auto fold = [&](R* v, const int cnt, const int ic0, const double scale) {
      constexpr int kS = kFoldMax | 1;
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int j = 0; j < kFoldMax; ++j)
        if (j < cnt) rec[lane * kS + j] = v[j];
      __builtin_amdgcn_wave_barrier();
      if (lane < cnt) {
        double s = 0.0;
#pragma unroll 8
        for (int i = 0; i < kWave; ++i) s += (double)rec[i * kS + lane];
        const int ic = ic0 + lane;
        acc[wid][ic >> 6][ic & (kWave - 1)] += s * scale;
      }
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int j = 0; j < kFoldMax; ++j)
        if (j < cnt) v[j] = (R)0;
    };

    auto flush = [&]() {
      if (nrec > 0) {
        // records written by other lanes are read here and the area is
        // reused right after: keep these LDS accesses in program order
        __builtin_amdgcn_wave_barrier();
        R xr[3] = {(R)0, (R)0, (R)0};
        R yr = (R)0;
        uint32_t rsteps = 0, rcens = 0;
        double rph = 0.0;
        if (lane < nrec) {
          R xe[DIM];
#pragma unroll
          for (int k = 0; k < DIM; ++k) xe[k] = rec[k * kWave + lane];
          const R y = rec[DIM * kWave + lane], z = rec[(DIM + 1) * kWave + lane];
          const uint32_t pr = rec_i[wid][0][lane], nr = rec_i[wid][1][lane];
          project<R, DIM>(D, xe, xr);
          const R gv = g_value_tp<R, DIM, TP>(P, tst, xr);
          const R phi = gv * y + z;
          const double ph = (double)phi;
          if constexpr (kWaveStats) {
            rph = ph;
            rsteps = nr & 0x7FFFFFFFu;
            rcens = nr >> 31;
          } else {
            wn += 1.0;
            const double d1 = ph - wmean;
            wmean += d1 / wn;
            wm2 += d1 * (ph - wmean);
            lsteps += (int64_t)(nr & 0x7FFFFFFFu);
            lcens += (int64_t)(nr >> 31);
          }
          if (dump_phi != nullptr) {
            const int64_t o = dump_off[node] + (int64_t)pr;
            dump_phi[o] = ph;
            if (dump_steps != nullptr) dump_steps[o] = (int64_t)(nr & 0x7FFFFFFFu);
          }
          if constexpr (ADJ) {
#pragma unroll
            for (int j = 0; j < NP; ++j) Br[j] -= phi * rec[(DIM + 2 + j) * kWave + lane];
#pragma unroll
            for (int t = 0; t < NT; ++t)
              if (t < P.g.n_terms) Gr[t] += y * TP::template term<R, DIM, FUN_G>(P, t, xr);
            yr = y;
          }
        }
        if constexpr (kWaveStats) {
          // the records' values, step and censoring counts into the
          // wavefront's item totals: a butterfly Welford merge over the
          // record lanes, then one Chan merge into the running triple
          double bn = lane < nrec ? 1.0 : 0.0, bm = rph, bq = 0.0;
          wave_welford(bn, bm, bq);
          const int64_t fs = wave_sum((int64_t)rsteps);
          const int64_t fc = (int64_t)__popcll(ballot(rcens != 0));
          if (lane == 0) {
            double an = wstat[wid][0], am = wstat[wid][1], aq = wstat[wid][2];
            chan_merge(an, am, aq, bn, bm, bq);
            wstat[wid][0] = an;
            wstat[wid][1] = am;
            wstat[wid][2] = aq;
            wcount[wid][0] += fs;
            wcount[wid][1] += fc;
          }
        }
        if constexpr (ADJ) {
          // g polynomial: column k gets the sum over the records of
          // Y monomial_k(X_tau).  Record lanes write their power rows, then
          // lane k % 64 sums monomial k over the records in FP64.
          if (P.g.poly_deg >= 0) {
            const int deg = P.g.poly_deg;
            __builtin_amdgcn_wave_barrier();
            if (lane < nrec) {
              R* row = rec + lane * kPwStride;
              R pa = yr;
              for (int e = 0; e <= deg; ++e) {
                row[e] = pa;
                pa *= xr[0];
              }
              if constexpr (DIM >= 2) {
                R pb = xr[1];
                for (int e = 1; e <= deg; ++e) {
                  row[deg + e] = pb;
                  pb *= xr[1];
                }
              }
              if constexpr (DIM >= 3) {
                R pc = xr[2];
                for (int e = 1; e <= deg; ++e) {
                  row[2 * deg + e] = pc;
                  pc *= xr[2];
                }
              }
              row[DIM * deg + 1] = (R)1;
            }
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int r = 0; r < kGSlots; ++r) {
              const int k = r * kWave + lane;
              if (k < ngm) {
                const uint32_t m = gmono[k];
                const int ra = (int)(m & 0xFFu), rb = (int)((m >> 8) & 0xFFu), rc = (int)(m >> 16);
                double sum = 0.0;
                for (int i = 0; i < nrec; ++i) {
                  const R* row = rec + i * kPwStride;
                  sum += (double)(row[ra] * row[rb] * row[rc]);
                }
                const int ic = 2 * NP + NT + k;
                acc[wid][ic >> 6][ic & (kWave - 1)] += sum;
              }
            }
          }
        }
        __builtin_amdgcn_wave_barrier();
        nrec = 0;
      }
      if constexpr (ADJ) {
        if constexpr (NP > 0) {
          fold(Fr, NP, 0, (double)dt);
          fold(Br, NP, NP, (double)dt);
        }
        if constexpr (NT > 0) fold(Gr, NT, 2 * NP, 1.0);
      }
    };

    for (;;) {
      // ---- stepping: refill_groups groups of GS::G Euler steps
      for (int gi = 0; gi < refill_groups; ++gi) {
        if (!__any(alive)) break;
        R z[GS::NZ];
        {
          const uint64_t blk0 = ((uint64_t)n * DIM) / NZr::kPerBlock;
#pragma unroll
          for (int b = 0; b < GS::NB; ++b) {
            const uint64_t blk = blk0 + (uint64_t)b;
            // opaque copies of the key: the round keys are rebuilt with
            // scalar adds at each use instead of living in registers
            uint32_t ka = k0, kb = k1;
            asm volatile("" : "+s"(ka), "+s"(kb));
            NZr::gen((uint32_t)blk, (uint32_t)((blk >> 32) & 0xFFFFFFu), path, (uint32_t)node, ka, kb,
                     &z[b * NZr::kPerBlock]);
          }
        }
#pragma unroll
        for (int s = 0; s < GS::G; ++s) {
          if constexpr (WOS) {
            // walk on spheres: jump by the distance to the boundary in the
            // direction of this jump's Gaussians, or stop inside the eps
            // shell.  Predicated, not branched (the branch's exec-mask
            // bookkeeping is scalar work, and the scalar unit bounds these
            // short steps): a lane that stops or is inactive jumps by a
            // radius of 0, an active one by the same operations.
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
          if constexpr (DFC < 0 && !TERMS && !ADJ) {
            // b = c = f = 0 (no polynomial, no terms): the pure-diffusion
            // step, predicated the same way (an inactive lane adds 0 z)
            const bool act = alive && n < max_steps;
            const R m = act ? sdt : (R)0;
#pragma unroll
            for (int k = 0; k < DIM; ++k) X[k] = X[k] + m * z[s * DIM + k];
            n += act ? 1u : 0u;
            const bool out = act && !inside<R, DIM>(Dt, X);
            alive = alive && !out;
            fin = fin || out;
            continue;
          }
          if (alive && n < max_steps) {
            R mono[NM > 0 ? NM : 1];
            if constexpr (DFC >= 0) monomials<R, DIM, DFC>(X, mono);
            R fv, cv;
            if constexpr (kLdsPoly) {
              const __attribute__((address_space(3))) R* lp = (const __attribute__((address_space(3))) R*)lpoly;
              fv = P.f.poly_deg >= 0 ? poly_dot_lds<R, NM>(lp + kNMp, mono) : (R)0;
              cv = P.c.poly_deg >= 0 ? poly_dot_lds<R, NM>(lp, mono) : (R)0;
            } else {
              fv = bcf_value<R, DIM, DFC, TERMS, TP, FUN_F>(P, tst, P.f, X, mono);
              cv = bcf_value<R, DIM, DFC, TERMS, TP, FUN_C>(P, tst, P.c, X, mono);
            }
            if constexpr (ADJ) {
#pragma unroll
              for (int t = 0; t < NT; ++t)
                if (t < P.f.n_terms) Fr[t] += TP::template term<R, DIM, FUN_F>(P, t, X) * Y;
              if constexpr (NM > 0) {
                if (P.f.poly_deg >= 0) {
#pragma unroll
                  for (int m = 0; m < NM; ++m) Fr[NT + m] += mono[m] * Y;
                }
              }
            }
            // terms known to vanish are skipped: X + 0 dt, Z + 0 and
            // Y exp(0) leave the same bits as evaluating them
            if (P.has_f) Z = Z + fv * Y * dt;
            if constexpr (ADJ) {
#pragma unroll
              for (int t = 0; t < NT; ++t) {
                if (t < P.c.n_terms) {
                  const R e = TP::template term<R, DIM, FUN_C>(P, t, X);
                  S[t] += e;
                  Br[t] += e * Z;
                }
              }
              if constexpr (NM > 0) {
                if (P.c.poly_deg >= 0) {
#pragma unroll
                  for (int m = 0; m < NM; ++m) {
                    S[NT + m] += mono[m];
                    Br[NT + m] += mono[m] * Z;
                  }
                }
              }
            }
            if (P.has_c) Y = Y * fexp(-cv * dt);
            if (P.has_b) {
              R bv[DIM];
              if constexpr (TERMS) {
                bv[0] = bcf_value<R, DIM, DFC, TERMS, TP, FUN_B0>(P, tst, P.b[0], X, mono);
                if constexpr (DIM >= 2) bv[1] = bcf_value<R, DIM, DFC, TERMS, TP, FUN_B1>(P, tst, P.b[1], X, mono);
                if constexpr (DIM >= 3) bv[2] = bcf_value<R, DIM, DFC, TERMS, TP, FUN_B2>(P, tst, P.b[2], X, mono);
              } else {
#pragma unroll
                for (int k = 0; k < DIM; ++k) bv[k] = bcf_value<R, DIM, DFC, false, TP, FUN_B0>(P, tst, P.b[k], X, mono);
              }
#pragma unroll
              for (int k = 0; k < DIM; ++k) X[k] = X[k] + bv[k] * dt + sdt * z[s * DIM + k];
            } else {
#pragma unroll
              for (int k = 0; k < DIM; ++k) X[k] = X[k] + sdt * z[s * DIM + k];
            }
            ++n;
            if (!inside<R, DIM>(Dt, X)) {
              alive = false;
              fin = true;
            }
          }
        }
      }
      if (alive && n >= max_steps) {
        alive = false;
        fin = true;
        // walk on spheres: a path already inside the eps shell exits normally
        cens = WOS ? (boundary_distance<R, DIM>(D, X) >= dt) : true;
      }

      // ---- park ended paths in LDS, refill their lanes with the item's next paths
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
#pragma unroll
          for (int j = 0; j < NP; ++j) rec[(DIM + 2 + j) * kWave + slot] = S[j];
          rec_i[wid][0][slot] = path;
          rec_i[wid][1][slot] = n | (cens ? 0x80000000u : 0u);
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
#pragma unroll
            for (int j = 0; j < NP; ++j) S[j] = (R)0;
          } else {
            path = pend;
          }
        }
      }
      if (!__any(alive) && !__any(fin)) break;
    }

    // ---- item results
    flush();
    if constexpr (kWaveStats) {
      wn = wstat[wid][0];
      wmean = wstat[wid][1];
      wm2 = wstat[wid][2];
      lsteps = wcount[wid][0];
      lcens = wcount[wid][1];
    } else {
      wave_welford(wn, wmean, wm2);
      lsteps = wave_sum(lsteps);
      lcens = wave_sum(lcens);
    }
    if (lane == 0 && istat != nullptr) {
      ItemStat st;
      st.mean = wmean;
      st.m2 = wm2;
      st.n = (int64_t)wn;
      st.steps = lsteps;
      st.censored = lcens;
      st.redrawn = 0;
      istat[it.slot] = st;
    }
    if constexpr (ADJ) {
      // row layout: [g terms NT | g poly nested ngm | f NP | c NP];
      // accumulator column ic: [f NP | c NP | g terms NT | g poly ngm]
      double* row = igrad + (size_t)it.slot * (size_t)grad_stride;
      const int ncols = 2 * NP + NT + ngm;
#pragma unroll
      for (int r = 0; r < kSlots; ++r) {
        const int ic = r * kWave + lane;
        if (ic < ncols) row[ic < 2 * NP ? NT + ngm + ic : ic - 2 * NP] = acc[wid][r][lane];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// FP64 baseline: one node per launch, one path per thread (grid-stride), each
// path run to its exit; Gaussians generated on demand one block at a time.
template <int DIM, int DFC, int LAYOUT>
__global__ void __launch_bounds__(kBlock)
k_walk_plain(const LinearParams P, int node, uint32_t n_paths, ItemStat* __restrict__ bstat,
             double* __restrict__ dump_phi, int64_t* __restrict__ dump_steps, int64_t dump_base) {
  using NZr = Normals<double, LAYOUT>;
  constexpr int PB = NZr::kPerBlock;
  const Dom<double> D = make_dom<double>(P);
  const Dom<double> Dt = make_test_dom<double>(P);
  double x0[DIM];
#pragma unroll
  for (int k = 0; k < DIM; ++k) x0[k] = P.nodes[(size_t)node * DIM + k];
  const bool node_in = inside<double, DIM>(Dt, x0);
  double wn = 0.0, wmean = 0.0, wm2 = 0.0;
  int64_t lsteps = 0, lcens = 0;
  for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < n_paths; p += gridDim.x * blockDim.x) {
    double X[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) X[k] = x0[k];
    double Y = 1.0, Z = 0.0;
    uint32_t n = 0;
    bool cens = false;
    if (node_in) {
      uint64_t cur = ~0ull;
      double zc[PB];
      for (;;) {
        if ((int64_t)n >= P.max_steps) { cens = true; break; }
        BCF<double, DIM, DFC> e;
        if constexpr (DFC >= 0) monomials<double, DIM, DFC>(X, e.mono);
        const double fv = fun_value<double, DIM, DFC>(P, P.f, X, e.mono);
        const double cv = fun_value<double, DIM, DFC>(P, P.c, X, e.mono);
        double bv[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) bv[k] = fun_value<double, DIM, DFC>(P, P.b[k], X, e.mono);
        Z = Z + fv * Y * P.dt;
        Y = Y * exp(-cv * P.dt);
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
          const uint64_t j = (uint64_t)n * DIM + k;
          const uint64_t blk = j / PB;
          if (blk != cur) {
            NZr::gen((uint32_t)blk, (uint32_t)((blk >> 32) & 0xFFFFFFu), p, (uint32_t)node, P.key0, P.key1, zc);
            cur = blk;
          }
          double zk = zc[0];
#pragma unroll
          for (int q = 1; q < PB; ++q) if ((int)(j % PB) == q) zk = zc[q];
          X[k] = X[k] + bv[k] * P.dt + P.sdt * zk;
        }
        ++n;
        if (!inside<double, DIM>(Dt, X)) break;
      }
    }
    double xp[3];
    project<double, DIM>(D, X, xp);
    const double phi = g_value<double, DIM>(P, xp) * Y + Z;
    wn += 1.0;
    const double d1 = phi - wmean;
    wmean += d1 / wn;
    wm2 += d1 * (phi - wmean);
    lsteps += n;
    lcens += cens ? 1 : 0;
    if (dump_phi != nullptr) {
      dump_phi[dump_base + p] = phi;
      if (dump_steps != nullptr) dump_steps[dump_base + p] = n;
    }
  }
  // block reduction: waves, then wave 0 merges the per-wave partials in order
  __shared__ double sn[kBlock / kWave], sm[kBlock / kWave], sq[kBlock / kWave];
  __shared__ int64_t ss[kBlock / kWave], sc[kBlock / kWave];
  wave_welford(wn, wmean, wm2);
  lsteps = wave_sum(lsteps);
  lcens = wave_sum(lcens);
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  if (lane == 0) { sn[wid] = wn; sm[wid] = wmean; sq[wid] = wm2; ss[wid] = lsteps; sc[wid] = lcens; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double n = 0.0, m = 0.0, q = 0.0;
    int64_t st = 0, ce = 0;
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) {
      chan_merge(n, m, q, sn[w], sm[w], sq[w]);
      st += ss[w];
      ce += sc[w];
    }
    ItemStat r;
    r.mean = m; r.m2 = q; r.n = (int64_t)n; r.steps = st; r.censored = ce; r.redrawn = 0;
    bstat[blockIdx.x] = r;
  }
}

// ---------------------------------------------------------------------------
// FP64 plain adjoint: one node per launch, one path per thread (grid covers
// the node's paths), the straightforward per-path tangents
//   F_j += m_j Y dt,  A_j += f Y dt S_j (before S moves),  S_j += m_j dt,
// and at the exit d phi/d f_j = F_j, d phi/d c_j = -g Y S_j - A_j,
// d phi/d g_k = Y G_k(X_tau).  Each block reduces its paths' derivatives
// into one row (layout as k_walk: [g terms NT | g poly nested | f NP | c NP])
// and its statistics into one ItemStat.
template <int DIM, int DFC, int LAYOUT, int NT>
__global__ void __launch_bounds__(kBlock)
k_walk_plain_adj(const LinearParams P, int node, uint32_t n_paths, ItemStat* __restrict__ bstat,
                 double* __restrict__ brow, int grad_stride) {
  using NZr = Normals<double, LAYOUT>;
  constexpr int PB = NZr::kPerBlock;
  constexpr int NM = GradedLex<DIM, DFC>::N;
  constexpr int NP = NT + NM;
  const Dom<double> D = make_dom<double>(P);
  const Dom<double> Dt = make_test_dom<double>(P);
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  double x0[DIM];
#pragma unroll
  for (int k = 0; k < DIM; ++k) x0[k] = P.nodes[(size_t)node * DIM + k];
  const bool node_in = inside<double, DIM>(Dt, x0);
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  const bool have = p < n_paths;

  double X[DIM];
#pragma unroll
  for (int k = 0; k < DIM; ++k) X[k] = x0[k];
  double Y = 1.0, Z = 0.0;
  uint32_t n = 0;
  bool cens = false;
  double F[NP > 0 ? NP : 1], S[NP > 0 ? NP : 1], A[NP > 0 ? NP : 1];
#pragma unroll
  for (int j = 0; j < NP; ++j) F[j] = S[j] = A[j] = 0.0;
  if (have && node_in) {
    uint64_t cur = ~0ull;
    double zc[PB];
    for (;;) {
      if ((int64_t)n >= P.max_steps) { cens = true; break; }
      BCF<double, DIM, DFC> e;
      if constexpr (DFC >= 0) monomials<double, DIM, DFC>(X, e.mono);
      const double fv = fun_value<double, DIM, DFC>(P, P.f, X, e.mono);
      const double cv = fun_value<double, DIM, DFC>(P, P.c, X, e.mono);
      const double fYdt = fv * Y * P.dt;
      const double Ydt = Y * P.dt;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        if (t < P.c.n_terms) {
          A[t] += fYdt * S[t];
          S[t] += term_value<double, DIM>(P.fac, P.c, t, X) * P.dt;
        }
        if (t < P.f.n_terms) F[t] += term_value<double, DIM>(P.fac, P.f, t, X) * Ydt;
      }
      if constexpr (DFC >= 0) {
        if (P.c.poly_deg >= 0) {
#pragma unroll
          for (int m = 0; m < NM; ++m) {
            A[NT + m] += fYdt * S[NT + m];
            S[NT + m] += e.mono[m] * P.dt;
          }
        }
        if (P.f.poly_deg >= 0) {
#pragma unroll
          for (int m = 0; m < NM; ++m) F[NT + m] += e.mono[m] * Ydt;
        }
      }
      double bv[DIM];
#pragma unroll
      for (int k = 0; k < DIM; ++k) bv[k] = fun_value<double, DIM, DFC>(P, P.b[k], X, e.mono);
      Z = Z + fv * Y * P.dt;
      Y = Y * exp(-cv * P.dt);
#pragma unroll
      for (int k = 0; k < DIM; ++k) {
        const uint64_t j = (uint64_t)n * DIM + k;
        const uint64_t blk = j / PB;
        if (blk != cur) {
          NZr::gen((uint32_t)blk, (uint32_t)((blk >> 32) & 0xFFFFFFu), p, (uint32_t)node, P.key0, P.key1, zc);
          cur = blk;
        }
        double zk = zc[0];
#pragma unroll
        for (int q = 1; q < PB; ++q) if ((int)(j % PB) == q) zk = zc[q];
        X[k] = X[k] + bv[k] * P.dt + P.sdt * zk;
      }
      ++n;
      if (!inside<double, DIM>(Dt, X)) break;
    }
  }
  double xp[3];
  project<double, DIM>(D, X, xp);
  const double gv = g_value<double, DIM>(P, xp);
  const double phi = gv * Y + Z;

  // block statistics: one sample per thread that has a path
  __shared__ double sn[kBlock / kWave], sm[kBlock / kWave], sq[kBlock / kWave], red[kBlock / kWave];
  __shared__ int64_t ss[kBlock / kWave], sc[kBlock / kWave];
  double wn = have ? 1.0 : 0.0, wmean = have ? phi : 0.0, wm2 = 0.0;
  int64_t lsteps = have ? (int64_t)n : 0, lcens = (have && cens) ? 1 : 0;
  wave_welford(wn, wmean, wm2);
  lsteps = wave_sum(lsteps);
  lcens = wave_sum(lcens);
  if (lane == 0) { sn[wid] = wn; sm[wid] = wmean; sq[wid] = wm2; ss[wid] = lsteps; sc[wid] = lcens; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double bn = 0.0, bm = 0.0, bq = 0.0;
    int64_t st = 0, ce = 0;
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) {
      chan_merge(bn, bm, bq, sn[w], sm[w], sq[w]);
      st += ss[w];
      ce += sc[w];
    }
    ItemStat r;
    r.mean = bm; r.m2 = bq; r.n = (int64_t)bn; r.steps = st; r.censored = ce; r.redrawn = 0;
    bstat[blockIdx.x] = r;
  }

  // derivative columns, one block sum each (waves in order)
  double* row = brow + (size_t)blockIdx.x * (size_t)grad_stride;
  auto put = [&](int col, double v) {
    const double s = wave_sum(have ? v : 0.0);
    __syncthreads();
    if (lane == 0) red[wid] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < (int)(blockDim.x / kWave); ++w) t += red[w];
      row[col] = t;
    }
  };
  int col = 0;
#pragma unroll
  for (int t = 0; t < NT; ++t) put(col + t, t < P.g.n_terms ? Y * term_value<double, DIM>(P.fac, P.g, t, xp) : 0.0);
  col += NT;
  if (P.g.poly_deg >= 0) {
    const int deg = P.g.poly_deg;
    double xa = Y;
    for (int a = 0; a <= deg; ++a) {
      double xb = xa;
      for (int b = 0; b <= (DIM >= 2 ? deg - a : 0); ++b) {
        double xc = xb;
        for (int c = 0; c <= (DIM >= 3 ? deg - a - b : 0); ++c) {
          put(col++, xc);
          if (DIM >= 3) xc *= xp[2];
        }
        if (DIM >= 2) xb *= xp[1];
      }
      xa *= xp[0];
    }
  }
#pragma unroll
  for (int j = 0; j < NP; ++j) put(col + j, F[j]);
  col += NP;
#pragma unroll
  for (int j = 0; j < NP; ++j) put(col + j, -gv * Y * S[j] - A[j]);
}

#ifndef __HIPCC_RTC__
// ---------------------------------------------------------------------------
// Launch of one k_walk instantiation, dispatched on dimension and on whether
// b, c, f have a polynomial part.
template <typename R, int DIM, int DFC, int LAYOUT, bool TERMS, bool ADJ, bool WOS = false>
static hipError_t launch_walk_t(const WalkLaunch& L, hipStream_t st) {
  hipLaunchKernelGGL((k_walk<R, DIM, DFC, LAYOUT, TERMS, ADJ, WOS>), dim3(L.grid), dim3(kBlock), 0, st, *L.P, L.items,
                     L.n_items, L.qhead, L.istat, L.igrad, L.grad_stride, L.dump_phi, L.dump_steps, L.dump_off,
                     L.refill_groups);
  return hipGetLastError();
}

template <typename R, int LAYOUT, bool TERMS, bool ADJ>
static hipError_t launch_walk_dim(const WalkLaunch& L, hipStream_t st) {
  const bool poly = L.dfc >= 0;
  switch (L.P->dim) {
    case 1:
      return poly ? launch_walk_t<R, 1, 3, LAYOUT, TERMS, ADJ>(L, st) : launch_walk_t<R, 1, -1, LAYOUT, TERMS, ADJ>(L, st);
    case 2:
      return poly ? launch_walk_t<R, 2, 3, LAYOUT, TERMS, ADJ>(L, st) : launch_walk_t<R, 2, -1, LAYOUT, TERMS, ADJ>(L, st);
    default:
      return poly ? launch_walk_t<R, 3, 3, LAYOUT, TERMS, ADJ>(L, st) : launch_walk_t<R, 3, -1, LAYOUT, TERMS, ADJ>(L, st);
  }
}

template <typename R, int LAYOUT, bool ADJ>
static hipError_t launch_walk_terms(const WalkLaunch& L, hipStream_t st) {
  return L.terms ? launch_walk_dim<R, LAYOUT, true, ADJ>(L, st) : launch_walk_dim<R, LAYOUT, false, ADJ>(L, st);
}

#endif  // __HIPCC_RTC__

}  // namespace pdd
