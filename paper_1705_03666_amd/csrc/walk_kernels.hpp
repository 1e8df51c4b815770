// Feynman-Kac walk kernels (Sec. 2.2, eqs. 2.7-2.9 in the elliptic
// pure-Dirichlet limit; Euler-Maruyama plus boundary test, Sec. 2.1).
//
//  k_walk<R, DIM, DFC, LAYOUT, NT, ADJ>  persistent batched kernel: every
//      wavefront pops work items (node, path range) from a device queue and
//      runs one path per lane; a lane whose path has exited takes the next
//      path index of the item ("refill"), so lanes stay busy while exit times
//      vary tenfold.  R = float: FP32 stepping / transforms; R = double: FP64.
//      With ADJ the same paths are re-simulated with pathwise tangents and the
//      derivative of each path value with respect to the coefficients of g, f
//      and c is accumulated per item (the exact derivative of the discrete
//      estimator).
//  k_walk_plain<DIM, DFC, LAYOUT>  the FP64 baseline: one node per launch,
//      one path per thread until it exits, block-level partial statistics.
//
// Path p of node i draws its Gaussians from Philox counters
// (block, stream 0 | block >> 32, p, i): the path is a pure function of
// (seed, i, p), independent of which lane or launch computes it.
#pragma once
#include <hip/hip_runtime.h>

#include "pdd_device.hpp"
#include "pdd_kernels.hpp"

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

// Per-lane tangent state of the adjoint (unused when ADJ is false).
template <typename R, int NT, int NM>
struct Tangents {
  static constexpr int NP = NT + NM;
  R F[NP > 0 ? NP : 1];   // d Z / d coef_f
  R S[NP > 0 ? NP : 1];   // sum of c-basis * dt
  R A[NP > 0 ? NP : 1];   // sum of f Y dt S (before the S update)
};

template <typename R, int DIM, int DFC, int LAYOUT, int NT, bool ADJ>
__global__ void __launch_bounds__(kBlock)
k_walk(const LinearParams P, const WorkItem* __restrict__ items, int n_items, uint32_t* __restrict__ qhead,
       ItemStat* __restrict__ istat, double* __restrict__ igrad, int grad_stride,
       double* __restrict__ dump_phi, int64_t* __restrict__ dump_steps, const int64_t* __restrict__ dump_off,
       int refill_groups) {
  using NZr = Normals<R, LAYOUT>;
  using GS = GroupShape<DIM, NZr::kPerBlock>;
  constexpr int NM = GradedLex<DIM, DFC>::N;
  constexpr int NP = NT + NM;
  constexpr int kGAcc = (GradedLex<3, kMaxPolyG>::N + kWave - 1) / kWave;

  const int lane = (int)(threadIdx.x & (kWave - 1));
  const int wid = (int)(threadIdx.x / kWave);
  __shared__ R rec_x[ADJ ? kBlock / kWave : 1][ADJ ? kWave : 1][3];
  __shared__ R rec_y[ADJ ? kBlock / kWave : 1][ADJ ? kWave : 1];
  // Per-item sums of the path derivatives, one private column per lane
  // (rows: f parameters, c parameters, generic g terms).  Keeping them in LDS
  // rather than registers leaves room for the per-path tangents.
  constexpr int kAccRows = ADJ ? 2 * NP + NT : 1;
  __shared__ R acc[ADJ ? kBlock / kWave : 1][kAccRows > 0 ? kAccRows : 1][ADJ ? kWave : 1];
  // Forward: exit records (x_tau[3], Y, Z) and (path, steps | censored << 31).
  __shared__ R frec[ADJ ? 1 : kBlock / kWave][ADJ ? 1 : kWave][5];
  __shared__ uint32_t frec_i[ADJ ? 1 : kBlock / kWave][ADJ ? 1 : kWave][2];

  const Dom<R> D = make_dom<R>(P);
  const R dt = dt_of<R>(P);
  const R sdt = sdt_of<R>(P);
  const uint32_t k0 = P.key0, k1 = P.key1;

  for (;;) {
    const uint32_t it_idx = pop_item(qhead);
    if (it_idx >= (uint32_t)n_items) break;
    const WorkItem it = items[it_idx];
    const int node = it.node;
    const uint32_t pend = it.p0 + it.count;

    R x0[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) x0[k] = to_r<R>(P.nodes[(size_t)node * DIM + k]);
    const bool node_in = inside<R, DIM>(D, x0);

    // lane state
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

    Tangents<R, NT, NM> T;
    double gacc[ADJ ? kGAcc : 1];
    int nrec = 0;
    int nfrec = 0;

    // Forward exit batch: lane l takes record l, evaluates g there, and folds
    // phi = g Y + Z into its own Welford triple (every path of the item
    // belongs to the same node, so any lane may take any path).
    auto flush_exits = [&]() {
      if constexpr (!ADJ) {
        if (nfrec == 0) return;
        // records written by other lanes are read here and the slots are
        // reused right after: keep these LDS accesses in program order
        __builtin_amdgcn_wave_barrier();
        if (lane < nfrec) {
          R xp[3] = {(R)0, (R)0, (R)0};
#pragma unroll
          for (int k = 0; k < DIM; ++k) xp[k] = frec[wid][lane][k];
          const R yr = frec[wid][lane][3], zr = frec[wid][lane][4];
          const uint32_t pr = frec_i[wid][lane][0], nr = frec_i[wid][lane][1];
          const double ph = (double)(g_value<R, DIM>(P, xp) * yr + zr);
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
        nfrec = 0;
      }
    };
    if constexpr (ADJ) {
#pragma unroll
      for (int j = 0; j < NP; ++j) T.F[j] = T.S[j] = T.A[j] = (R)0;
      for (int j = 0; j < kAccRows; ++j) acc[wid][j][lane] = (R)0;
#pragma unroll
      for (int r = 0; r < kGAcc; ++r) gacc[r] = 0.0;
    }

    // g-polynomial gradient: the sum over exited paths of Y * monomial(X_tau),
    // batched through LDS records (one record per lane), reduced monomial by
    // monomial; lane (j % 64) keeps nested-order monomial j.
    auto flush_records = [&]() {
      if constexpr (ADJ) {
        if (nrec == 0 || P.g.poly_deg < 0) { nrec = 0; return; }
        __builtin_amdgcn_wave_barrier();
        const bool have = lane < nrec;
        R xr[3] = {(R)0, (R)0, (R)0};
        R yr = (R)0;
        if (have) {
#pragma unroll
          for (int k = 0; k < DIM; ++k) xr[k] = rec_x[wid][lane][k];
          yr = rec_y[wid][lane];
        }
        const int deg = P.g.poly_deg;
        int idx = 0;
        R xa = yr;
        for (int a = 0; a <= deg; ++a) {
          R xb = xa;
          for (int b = 0; b <= (DIM >= 2 ? deg - a : 0); ++b) {
            R xc = xb;
            for (int c = 0; c <= (DIM >= 3 ? deg - a - b : 0); ++c) {
              const double s = wave_sum((double)xc);
              const int slot = idx / kWave;
              if (lane == (idx & (kWave - 1))) {
#pragma unroll
                for (int r = 0; r < kGAcc; ++r) if (r == slot) gacc[r] += s;
              }
              ++idx;
              if (DIM >= 3) xc *= xr[2];
            }
            if (DIM >= 2) xb *= xr[1];
          }
          xa *= xr[0];
        }
        __builtin_amdgcn_wave_barrier();
        nrec = 0;
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
            NZr::gen((uint32_t)blk, (uint32_t)((blk >> 32) & 0xFFFFFFu), path, (uint32_t)node, k0, k1,
                     &z[b * NZr::kPerBlock]);
          }
        }
#pragma unroll
        for (int s = 0; s < GS::G; ++s) {
          if (alive) {
            if ((int64_t)n >= P.max_steps) {
              alive = false;
              fin = true;
              cens = true;
            } else {
              BCF<R, DIM, DFC> e;
              if constexpr (DFC >= 0) monomials<R, DIM, DFC>(X, e.mono);
              const R fv = fun_value<R, DIM, DFC>(P, P.f, X, e.mono);
              const R cv = fun_value<R, DIM, DFC>(P, P.c, X, e.mono);
              if constexpr (ADJ) {
                const R fYdt = fv * Y * dt;
                const R Ydt = Y * dt;
                // generic terms of c and f, then their polynomial parts
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                  if (t < P.c.n_terms) {
                    T.A[t] += fYdt * T.S[t];
                    T.S[t] += term_value<R, DIM>(P.fac, P.c, t, X) * dt;
                  }
                  if (t < P.f.n_terms) T.F[t] += term_value<R, DIM>(P.fac, P.f, t, X) * Ydt;
                }
                if constexpr (DFC >= 0) {
                  if (P.c.poly_deg >= 0) {
#pragma unroll
                    for (int m = 0; m < NM; ++m) {
                      T.A[NT + m] += fYdt * T.S[NT + m];
                      T.S[NT + m] += e.mono[m] * dt;
                    }
                  }
                  if (P.f.poly_deg >= 0) {
#pragma unroll
                    for (int m = 0; m < NM; ++m) T.F[NT + m] += e.mono[m] * Ydt;
                  }
                }
              }
              Z = Z + fv * Y * dt;
              Y = Y * fexp(-cv * dt);
              R bv[DIM];
#pragma unroll
              for (int k = 0; k < DIM; ++k) bv[k] = fun_value<R, DIM, DFC>(P, P.b[k], X, e.mono);
#pragma unroll
              for (int k = 0; k < DIM; ++k) X[k] = X[k] + bv[k] * dt + sdt * z[s * DIM + k];
              ++n;
              if (!inside<R, DIM>(D, X)) {
                alive = false;
                fin = true;
              }
            }
          }
        }
      }

      const uint64_t fmask = ballot(fin);
      if (fmask == 0) {
        if (!__any(alive)) break;
        continue;
      }

      // ---- exits.  Forward: park (exit point, Y, Z, path, steps) in LDS and
      // evaluate g for 64 of them at a time, one per lane.  Adjoint: the
      // tangents need g at once, so the exiting lanes evaluate it here.
      if constexpr (!ADJ) {
        const int nf = __popcll(fmask);
        if (nfrec + nf > kWave) flush_exits();
        if (fin) {
          R xp[3];
          project<R, DIM>(D, X, xp);
          const int slot = nfrec + lane_rank(fmask);
#pragma unroll
          for (int k = 0; k < DIM; ++k) frec[wid][slot][k] = xp[k];
          frec[wid][slot][3] = Y;
          frec[wid][slot][4] = Z;
          frec_i[wid][slot][0] = path;
          frec_i[wid][slot][1] = n | (cens ? 0x80000000u : 0u);
        }
        nfrec += nf;
      }
      if constexpr (ADJ) {
        const int nf = __popcll(fmask);
        if (nrec + nf > kWave) flush_records();
      }
      if (ADJ && fin) {
        R xp[3];
        project<R, DIM>(D, X, xp);
        const R gv = g_value<R, DIM>(P, xp);
        const R phi = gv * Y + Z;
        const double ph = (double)phi;
        wn += 1.0;
        const double d1 = ph - wmean;
        wmean += d1 / wn;
        wm2 += d1 * (ph - wmean);
        lsteps += (int64_t)n;
        lcens += cens ? 1 : 0;
        if (dump_phi != nullptr) {
          const int64_t o = dump_off[node] + (int64_t)path;
          dump_phi[o] = ph;
          if (dump_steps != nullptr) dump_steps[o] = (int64_t)n;
        }
        if constexpr (ADJ) {
#pragma unroll
          for (int j = 0; j < NP; ++j) {
            acc[wid][j][lane] += T.F[j];
            acc[wid][NP + j][lane] += -gv * Y * T.S[j] - T.A[j];
          }
#pragma unroll
          for (int t = 0; t < NT; ++t)
            if (t < P.g.n_terms) acc[wid][2 * NP + t][lane] += Y * term_value<R, DIM>(P.fac, P.g, t, xp);
          const int slot = nrec + lane_rank(fmask);
#pragma unroll
          for (int k = 0; k < DIM; ++k) rec_x[wid][slot][k] = xp[k];
          rec_y[wid][slot] = Y;
        }
      }
      if constexpr (ADJ) nrec += __popcll(fmask);

      // ---- refill finished lanes with the next paths of the item
      {
        const uint32_t np = cursor + (uint32_t)lane_rank(fmask);
        cursor += (uint32_t)__popcll(fmask);
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
            if constexpr (ADJ) {
#pragma unroll
              for (int j = 0; j < NP; ++j) T.F[j] = T.S[j] = T.A[j] = (R)0;
            }
          } else {
            path = pend;
          }
        }
      }
      if (!__any(alive) && !__any(fin)) break;
    }

    // ---- item results
    if constexpr (ADJ) flush_records();
    if constexpr (!ADJ) flush_exits();
    wave_welford(wn, wmean, wm2);
    lsteps = wave_sum(lsteps);
    lcens = wave_sum(lcens);
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
      double* row = igrad + (size_t)it.slot * (size_t)grad_stride;
      // row layout: [g terms NT | g poly nested (grad_stride budget) | f NP | c NP]
      int col = 0;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const double v = wave_sum((double)acc[wid][2 * NP + t][lane]);
        if (lane == 0) row[col + t] = v;
      }
      col += NT;
      const int ngm = P.g.poly_deg >= 0 ? P.g.n_mono : 0;
#pragma unroll
      for (int r = 0; r < kGAcc; ++r) {
        const int j = r * kWave + lane;
        if (j < ngm) row[col + j] = gacc[r];
      }
      col += ngm;
#pragma unroll
      for (int j = 0; j < NP; ++j) {
        const double v = wave_sum((double)acc[wid][j][lane]);
        if (lane == 0) row[col + j] = v;
      }
      col += NP;
#pragma unroll
      for (int j = 0; j < NP; ++j) {
        const double v = wave_sum((double)acc[wid][NP + j][lane]);
        if (lane == 0) row[col + j] = v;
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
  double x0[DIM];
#pragma unroll
  for (int k = 0; k < DIM; ++k) x0[k] = P.nodes[(size_t)node * DIM + k];
  const bool node_in = inside<double, DIM>(D, x0);
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
        if (!inside<double, DIM>(D, X)) break;
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

}  // namespace pdd
