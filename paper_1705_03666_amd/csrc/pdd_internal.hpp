// Structures shared by the host layer (capi.cpp) and the HIP kernels.
#pragma once
#ifdef __HIPCC_RTC__
// runtime compilation: the fixed-width types come with the compiler's own headers
typedef __hip_internal::int32_t int32_t;
typedef __hip_internal::uint32_t uint32_t;
typedef __hip_internal::int64_t int64_t;
typedef __hip_internal::uint64_t uint64_t;
#else
#include <stdint.h>
#endif

namespace pdd {

constexpr int kWave = 64;
constexpr int kBlock = 256;                 // 4 waves per workgroup
constexpr int kMaxFactors = 4;
constexpr int kMaxPolyBCF = 3;              // dense-polynomial degree limit for b, c, f
constexpr int kMaxPolyG = 8;                // dense-polynomial degree limit for g and psi
constexpr int kAdjTerms = 4;                // generic terms of g, f, c with tangents in the adjoint
constexpr int kMaxTerms = 64;

enum : int { FN_POW = 0, FN_EXP = 1, FN_SIN = 2, FN_COS = 3, FN_TANH = 4 };
enum : int { DOM_BOX = 0, DOM_BALL = 1, DOM_FREE = 2 };
enum : int { RNG_PAIR52 = 0, RNG_QUAD24 = 1 };

// Factor fn(a x[dim] + b)^power, in both precisions.
struct DevFactor {
  int32_t fn, dim, power, pad;
  float af, bf;
  double ad, bd;
};

// Where a function's data live inside the staged tables.  Coefficients are in
// one table (double and float copies); the dense polynomial of b, c, f is in
// graded-lex order, that of g and psi in "nested" order
// (for a: for b: for c, total degree <= deg) so that it can be evaluated by
// three running products.
struct DevFun {
  int32_t n_terms, n_factors, fac_off, coef_off;
  int32_t poly_deg, n_mono, poly_off, pad;
};

struct LinearParams {
  int32_t dim, dom_kind, layout, n_fac;
  double lo[3], hi[3], ctr[3], rad, rad2;
  float lof[3], hif[3], ctrf[3], radf, rad2f;
  double dt, sdt;                 // sdt = sigma * sqrt(dt)
  float dtf, sdtf;
  int64_t max_steps;
  uint32_t key0, key1;
  int32_t has_b, has_c, has_f, pad_flags;   // b, c, f not identically zero
  // domain of the exit test (D itself, or D shrunk for the boundary-corrected scheme)
  double tlo[3], thi[3], trad2;
  float tlof[3], thif[3], trad2f;
  DevFun b[3], c, f, g;
  const DevFactor* fac;
  const double* cd;
  const float* cf;
  const double* nodes;
};

struct BranchParams {
  int32_t dim, max_segments, label_base, n_fac;
  double sigma, beta, T;
  float sigmaf, betaf, Tf, inv_betaf;
  double alpha[5], q[5], ratio[5], qcum[5];
  float qcumf[5], pad1[3];
  // The offspring law in compact form: the n_cls classes with q > 0 in
  // increasing order, class j drawn when thr[j-1] <= u < thr[j] (thr[-1] = 0,
  // the last class for every u beyond), with its size and mark alpha / q.
  // thr[j] for j >= n_cls - 1 is +infinity, so the class index is the
  // number of thresholds at or below u.
  int32_t n_cls, pad2;
  int32_t cls[5], pad3;
  float thrf[4];
  double thr[4];
  double mark[5];
  uint32_t key0, key1;
  DevFun psi;
  const DevFactor* fac;
  const double* cd;
  const float* cf;
  const double* points;
};

// Dirichlet boundary and output times of the branching estimator with a
// boundary (eq. 3.2, Algorithm 3.1).  g is evaluated at (x, s): a factor
// whose coordinate index equals dim reads the time argument s.
constexpr int kMaxTimes = 12;
struct BranchBoundary {
  int32_t dom_kind, n_times;
  double lo[3], hi[3], ctr[3], rad, rad2;
  float lof[3], hif[3], ctrf[3], radf, rad2f;
  double dt;
  float dtf, pad0;
  double shift;                  // 0, or c0 of the per-sub-step boundary correction
  float shiftf, pad1;
  double times[kMaxTimes];
  float timesf[kMaxTimes];
  DevFun g;
};

// One unit of work for a wavefront: `count` consecutive paths (trees) of one
// node starting at path index p0.  `slot` is the item's position in
// node-major order, where its partial result is written.
struct WorkItem {
  int32_t node;
  uint32_t p0;
  uint32_t count;
  int32_t slot;
};

// Partial statistics of one work item (Welford triple + counters).
struct ItemStat {
  double mean, m2;
  int64_t n, steps, censored, redrawn;
};

// Copy job of the staging kernel.  With dst == nullptr it fills the staged
// coefficient tables: cd[dst_off + k] = src[perm ? perm[k] : k] (and the FP32
// shadow cf); otherwise it copies dst[k] = src[k] (node coordinates).
struct StageJob {
  const double* src;
  double* dst;
  int32_t dst_off, count, perm_off, pad;
};

// The caller's per-call buffers that the reduction kernels write or read.
// They live in one small device block that is rewritten before every launch,
// so a cached graph plan serves calls whose buffers differ.
struct CallPtrs {
  void* out;          // pdd_node_stat [n_nodes] (branching with a boundary: [n_times][n_nodes])
  const double* w;    // adjoint weights [n_nodes]
  double* jac;        // value+Jacobian output [n_nodes][jac_ld]
  double* grad[6];    // gradient destinations: g coef, g poly, f coef, f poly, c coef, c poly
};

}  // namespace pdd
