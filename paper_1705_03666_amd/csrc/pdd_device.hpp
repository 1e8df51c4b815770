// Device building blocks: counter-based Philox4x32-10, uniform lattices and
// Box-Muller, coefficient-function evaluation, domain test / projection and
// wavefront reductions.  Everything is a header so the compiler can inline it
// into each kernel instantiation.
#pragma once
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#include <stdint.h>
#endif

#include "pdd_internal.hpp"

namespace pdd {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 products
// and xors.  The key (the seed) is uniform across a wavefront, so the key
// schedule stays in scalar registers.  The three-way xors are single
// three-input bitwise operations (truth table 0x96 = a ^ b ^ c).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3,
                                              uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
    const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// ---------------------------------------------------------------------------
// Uniforms on open lattices and Gaussians.
//   QUAD24: u = (2 (w >> 9) + 1) 2^-24 (exact in FP32)
//   PAIR52: u = (2 k + 1) 2^-53, k = (w_hi << 20) | (w_lo >> 12) (exact in FP64)
// Box-Muller: z0 = r cos(2 pi u_b), z1 = r sin(2 pi u_b), r = sqrt(-2 ln u_a).
__device__ __forceinline__ float u24f(uint32_t w) {
  // 0x3F800000 | (w >> 9) is the float 1 + (w >> 9) 2^-23 in [1, 2) (one
  // funnel shift of 0x7F:w); subtracting 1 - 2^-24 is exact and leaves
  // (2 (w >> 9) + 1) 2^-24.
  const uint32_t bits = __builtin_amdgcn_alignbit(0x7Fu, w, 9);
  return __builtin_bit_cast(float, bits) - 0x1.fffffep-1f;
}
__device__ __forceinline__ double u24d(uint32_t w) {
  return (double)(w >> 9) * 0x1p-23 + 0x1p-24;
}
__device__ __forceinline__ double u52d(uint32_t whi, uint32_t wlo) {
  const uint64_t k = ((uint64_t)whi << 20) | (uint64_t)(wlo >> 12);
  return (double)k * 0x1p-52 + 0x1p-53;
}

// FP32 Box-Muller on the hardware transcendental units: v_log_f32 is log2,
// v_sin/v_cos_f32 take their argument in revolutions, so 2 pi u needs no
// multiply.  -2 ln u = -2 ln2 log2 u.
__device__ __forceinline__ void box_muller_f(float ua, float ub, float& z0, float& z1) {
  const float r = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(ua));
  z0 = r * __builtin_amdgcn_cosf(ub);
  z1 = r * __builtin_amdgcn_sinf(ub);
}
__device__ __forceinline__ void box_muller_d(double ua, double ub, double& z0, double& z1) {
  const double r = sqrt(-2.0 * log(ua));
  double s, c;
  sincos(2.0 * 3.14159265358979323846 * ub, &s, &c);
  z0 = r * c;
  z1 = r * s;
}

template <typename R, int LAYOUT>
struct Normals;

template <>
struct Normals<float, RNG_QUAD24> {
  static constexpr int kPerBlock = 4;
  __device__ __forceinline__ static void gen(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                             uint32_t k1, float* z) {
    philox4x32_10(c0, c1, c2, c3, k0, k1);
    box_muller_f(u24f(c0), u24f(c1), z[0], z[1]);
    box_muller_f(u24f(c2), u24f(c3), z[2], z[3]);
  }
};
template <>
struct Normals<double, RNG_QUAD24> {
  static constexpr int kPerBlock = 4;
  __device__ __forceinline__ static void gen(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                             uint32_t k1, double* z) {
    philox4x32_10(c0, c1, c2, c3, k0, k1);
    box_muller_d(u24d(c0), u24d(c1), z[0], z[1]);
    box_muller_d(u24d(c2), u24d(c3), z[2], z[3]);
  }
};
template <>
struct Normals<double, RNG_PAIR52> {
  static constexpr int kPerBlock = 2;
  __device__ __forceinline__ static void gen(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                             uint32_t k1, double* z) {
    philox4x32_10(c0, c1, c2, c3, k0, k1);
    box_muller_d(u52d(c0, c1), u52d(c2, c3), z[0], z[1]);
  }
};

// ---------------------------------------------------------------------------
// Elementary functions per precision.  FP32 uses the hardware exp2 / sin / cos
// units (inputs here stay far inside their valid ranges); FP64 uses the
// accurate library routines.
__device__ __forceinline__ float fexp(float x) { return __builtin_amdgcn_exp2f(x * 1.4426950408889634f); }
__device__ __forceinline__ double fexp(double x) { return exp(x); }
__device__ __forceinline__ float fsin(float x) { return __builtin_amdgcn_sinf(x * 0.15915494309189535f); }
__device__ __forceinline__ double fsin(double x) { return sin(x); }
__device__ __forceinline__ float fcos(float x) { return __builtin_amdgcn_cosf(x * 0.15915494309189535f); }
__device__ __forceinline__ double fcos(double x) { return cos(x); }
__device__ __forceinline__ float ftanh(float x) {
  // tanh x = 1 - 2 / (e^{2x} + 1); saturates correctly at both ends.
  const float e = __builtin_amdgcn_exp2f(x * 2.8853900817779268f);
  return 1.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f);
}
__device__ __forceinline__ double ftanh(double x) { return tanh(x); }

// Read-only tables (factor records, coefficients) are read through the
// constant address space, which compiles to scalar loads: the records are
// wave-uniform, so their fields land in scalar registers and the switch over
// the factor's function becomes a uniform branch.  The empty asm statement
// hides the table address from the optimiser, so the loads stay next to
// their use instead of being hoisted out of the stepping loop into scalar
// registers that would then spill.
#define PDD_CONST_AS __attribute__((address_space(4)))

template <typename T>
__device__ __forceinline__ const T PDD_CONST_AS* const_table(const T* p) {
  uint64_t a = reinterpret_cast<uint64_t>(p);
  asm volatile("" : "+s"(a));
  return (const T PDD_CONST_AS*)a;
}

template <typename R>
__device__ __forceinline__ R fac_a(const DevFactor& f);
template <>
__device__ __forceinline__ float fac_a<float>(const DevFactor& f) { return f.af; }
template <>
__device__ __forceinline__ double fac_a<double>(const DevFactor& f) { return f.ad; }
template <typename R>
__device__ __forceinline__ R fac_b(const DevFactor& f);
template <>
__device__ __forceinline__ float fac_b<float>(const DevFactor& f) { return f.bf; }
template <>
__device__ __forceinline__ double fac_b<double>(const DevFactor& f) { return f.bd; }

template <typename R>
__device__ __forceinline__ R coef_at(const double* __restrict__ cd, const float* __restrict__ cf, int i);
template <>
__device__ __forceinline__ float coef_at<float>(const double* __restrict__, const float* __restrict__ cf, int i) {
  return cf[i];
}
template <>
__device__ __forceinline__ double coef_at<double>(const double* __restrict__ cd, const float* __restrict__, int i) {
  return cd[i];
}

// Coordinate d of x (DIM coordinates; DIM = 4 when a time argument follows
// three space coordinates).
template <typename R, int DIM>
__device__ __forceinline__ R pick(const R* x, int d) {
  if (DIM == 1) return x[0];
  if (DIM == 2) return d == 0 ? x[0] : x[1];
  if (DIM == 3) return d == 0 ? x[0] : (d == 1 ? x[1] : x[2]);
  return d == 0 ? x[0] : (d == 1 ? x[1] : (d == 2 ? x[2] : x[3]));
}

// One factor.  The factor record is wave-uniform (scalar loads), so the switch
// is a uniform branch.
template <typename R, int DIM>
__device__ __forceinline__ R factor_value(const DevFactor& fa, const R* x) {
  const R s = fac_a<R>(fa) * pick<R, DIM>(x, fa.dim) + fac_b<R>(fa);
  R v;
  switch (fa.fn) {
    case FN_EXP: v = fexp(s); break;
    case FN_SIN: v = fsin(s); break;
    case FN_COS: v = fcos(s); break;
    case FN_TANH: v = ftanh(s); break;
    default: v = s; break;
  }
  R r = (R)1;
  for (int k = 0; k < fa.power; ++k) r *= v;
  return r;
}

// factor_value with the function and the power fixed at compile time (the
// form used by problem-specialised kernels): the same operations in the same
// order, so it returns the same bits.
template <typename R, int DIM, int FN, int POW>
__device__ __forceinline__ R factor_fixed(const R* x, int d, R a, R b) {
  const R s = a * pick<R, DIM>(x, d) + b;
  R v;
  if constexpr (FN == FN_EXP) v = fexp(s);
  else if constexpr (FN == FN_SIN) v = fsin(s);
  else if constexpr (FN == FN_COS) v = fcos(s);
  else if constexpr (FN == FN_TANH) v = ftanh(s);
  else v = s;
  R r = (R)1;
#pragma unroll
  for (int k = 0; k < POW; ++k) r *= v;
  return r;
}

// Product of the factors of term t (without its coefficient).
template <typename R, int DIM>
__device__ __forceinline__ R term_value(const DevFactor* __restrict__ fac, const DevFun& F, int t, const R* x) {
  R v = (R)1;
  const DevFactor PDD_CONST_AS* tf = const_table(fac) + F.fac_off + t * F.n_factors;
  for (int j = 0; j < F.n_factors; ++j) {
    DevFactor fa;
    fa.fn = tf[j].fn;
    fa.dim = tf[j].dim;
    fa.power = tf[j].power;
    fa.af = tf[j].af;
    fa.bf = tf[j].bf;
    fa.ad = tf[j].ad;
    fa.bd = tf[j].bd;
    v *= factor_value<R, DIM>(fa, x);
  }
  return v;
}

template <typename R>
__device__ __forceinline__ R coef_const(const double* __restrict__ cd, const float* __restrict__ cf, int i);
template <>
__device__ __forceinline__ float coef_const<float>(const double* __restrict__, const float* __restrict__ cf, int i) {
  return const_table(cf)[i];
}
template <>
__device__ __forceinline__ double coef_const<double>(const double* __restrict__ cd, const float* __restrict__, int i) {
  return const_table(cd)[i];
}

template <typename R, int DIM>
__device__ __forceinline__ R terms_sum(const DevFactor* __restrict__ fac, const double* __restrict__ cd,
                                       const float* __restrict__ cf, const DevFun& F, const R* x) {
  R s = (R)0;
  for (int t = 0; t < F.n_terms; ++t) s += coef_const<R>(cd, cf, F.coef_off + t) * term_value<R, DIM>(fac, F, t, x);
  return s;
}

// Dense polynomial of runtime degree, coefficients in nested order
// (a outer, b middle, c inner), evaluated with running products.
template <typename R, int DIM>
__device__ __forceinline__ R poly_nested(const double* __restrict__ cd, const float* __restrict__ cf, int deg,
                                         int off, const R* x) {
  R s = (R)0;
  int idx = off;
  R xa = (R)1;
  for (int a = 0; a <= deg; ++a) {
    if (DIM == 1) {
      s += coef_at<R>(cd, cf, idx++) * xa;
    } else {
      R xb = xa;
      for (int b = 0; b <= deg - a; ++b) {
        if (DIM == 2) {
          s += coef_at<R>(cd, cf, idx++) * xb;
        } else {
          R xc = xb;
          for (int c = 0; c <= deg - a - b; ++c) {
            s += coef_at<R>(cd, cf, idx++) * xc;
            xc *= x[2];
          }
        }
        xb *= x[1];
      }
    }
    xa *= x[0];
  }
  return s;
}

// Graded-lexicographic monomial table of total degree <= D in DIM variables,
// built at compile time so that fully unrolled loops index registers only.
constexpr int binom(int n, int k) {
  int r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}
template <int DIM, int D>
struct GradedLex {
  static constexpr int N = D < 0 ? 0 : binom(D + DIM, DIM);
  int e[N > 0 ? N : 1][3];
  constexpr GradedLex() : e{} {
    int m = 0;
    for (int k = 0; k <= D; ++k) {
      if (DIM == 1) {
        e[m][0] = k; e[m][1] = 0; e[m][2] = 0; ++m;
      } else if (DIM == 2) {
        for (int a = k; a >= 0; --a) { e[m][0] = a; e[m][1] = k - a; e[m][2] = 0; ++m; }
      } else {
        for (int a = k; a >= 0; --a)
          for (int b = k - a; b >= 0; --b) { e[m][0] = a; e[m][1] = b; e[m][2] = k - a - b; ++m; }
      }
    }
  }
};

// All monomials of degree <= D at x, graded-lex order.  Powers of unused
// coordinates are the constant 1, which the compiler folds away.
template <typename R, int DIM, int D>
__device__ __forceinline__ void monomials(const R* x, R* mono) {
  constexpr GradedLex<DIM, D> T{};
  R p[3][D + 1];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    p[k][0] = (R)1;
#pragma unroll
    for (int j = 1; j <= D; ++j) p[k][j] = (k < DIM) ? p[k][j - 1] * x[k < DIM ? k : 0] : (R)1;
  }
#pragma unroll
  for (int m = 0; m < GradedLex<DIM, D>::N; ++m) mono[m] = p[0][T.e[m][0]] * p[1][T.e[m][1]] * p[2][T.e[m][2]];
}

// ---------------------------------------------------------------------------
// Domain: open box or ball; a boundary point counts as outside.
template <typename R>
struct Dom {
  int kind;
  R lo[3], hi[3], ctr[3], rad, rad2;
};

template <typename R>
__device__ __forceinline__ Dom<R> make_dom(const LinearParams& P);
template <>
__device__ __forceinline__ Dom<float> make_dom<float>(const LinearParams& P) {
  Dom<float> D;
  D.kind = P.dom_kind;
  for (int k = 0; k < 3; ++k) { D.lo[k] = P.lof[k]; D.hi[k] = P.hif[k]; D.ctr[k] = P.ctrf[k]; }
  D.rad = P.radf;
  D.rad2 = P.rad2f;
  return D;
}
template <>
__device__ __forceinline__ Dom<double> make_dom<double>(const LinearParams& P) {
  Dom<double> D;
  D.kind = P.dom_kind;
  for (int k = 0; k < 3; ++k) { D.lo[k] = P.lo[k]; D.hi[k] = P.hi[k]; D.ctr[k] = P.ctr[k]; }
  D.rad = P.rad;
  D.rad2 = P.rad2;
  return D;
}

// Domain of the exit test: D, or D shrunk for the boundary-corrected scheme
// (only the fields the test reads: kind, lo, hi, ctr, rad2).
template <typename R>
__device__ __forceinline__ Dom<R> make_test_dom(const LinearParams& P);
template <>
__device__ __forceinline__ Dom<float> make_test_dom<float>(const LinearParams& P) {
  Dom<float> D;
  D.kind = P.dom_kind;
  for (int k = 0; k < 3; ++k) { D.lo[k] = P.tlof[k]; D.hi[k] = P.thif[k]; D.ctr[k] = P.ctrf[k]; }
  D.rad = P.radf;
  D.rad2 = P.trad2f;
  return D;
}
template <>
__device__ __forceinline__ Dom<double> make_test_dom<double>(const LinearParams& P) {
  Dom<double> D;
  D.kind = P.dom_kind;
  for (int k = 0; k < 3; ++k) { D.lo[k] = P.tlo[k]; D.hi[k] = P.thi[k]; D.ctr[k] = P.ctr[k]; }
  D.rad = P.rad;
  D.rad2 = P.trad2;
  return D;
}

template <typename R, int DIM>
__device__ __forceinline__ bool inside(const Dom<R>& D, const R* x) {
  if (D.kind == DOM_BOX) {
    bool in = true;
#pragma unroll
    for (int k = 0; k < DIM; ++k) in = in && (x[k] > D.lo[k]) && (x[k] < D.hi[k]);
    return in;
  }
  R r2 = (R)0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    const R d = x[k] - D.ctr[k];
    r2 += d * d;
  }
  return r2 < D.rad2;
}

// Distance from x to the boundary of D (negative outside): ball R - |x - c|,
// box min_k min(x_k - lo_k, hi_k - x_k).  FP64: every product and sum rounded
// on its own (no fused multiply-add), so that walk-on-spheres paths, whose
// jumps amplify rounding differences, follow the oracle's arithmetic exactly.
template <typename R, int DIM>
__device__ __forceinline__ R boundary_distance(const Dom<R>& D, const R* x) {
  if constexpr (sizeof(R) == 8) {
#pragma clang fp contract(off)
    if (D.kind == DOM_BOX) {
      R m = x[0] - D.lo[0];
      m = fmin(m, D.hi[0] - x[0]);
#pragma unroll
      for (int k = 1; k < DIM; ++k) {
        m = fmin(m, x[k] - D.lo[k]);
        m = fmin(m, D.hi[k] - x[k]);
      }
      return m;
    }
    R r2 = (R)0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      const R d = x[k] - D.ctr[k];
      r2 += d * d;
    }
    return D.rad - sqrt(r2);
  }
  if (D.kind == DOM_BOX) {
    R m = x[0] - D.lo[0];
    m = fmin(m, D.hi[0] - x[0]);
#pragma unroll
    for (int k = 1; k < DIM; ++k) {
      m = fmin(m, x[k] - D.lo[k]);
      m = fmin(m, D.hi[k] - x[k]);
    }
    return m;
  }
  R r2 = (R)0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    const R d = x[k] - D.ctr[k];
    r2 += d * d;
  }
  return D.rad - sqrt(r2);
}

// |z|^2 of one jump's Gaussians (FP64 without fused multiply-add, as above).
template <typename R, int DIM>
__device__ __forceinline__ R sum_squares(const R* z) {
  if constexpr (sizeof(R) == 8) {
#pragma clang fp contract(off)
    R s = (R)0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) s += z[k] * z[k];
    return s;
  }
  R s = (R)0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) s += z[k] * z[k];
  return s;
}

// x += r z / |z| (z2 = |z|^2): FP64 in the order r (z_k / |z|) with every
// operation rounded on its own (IEEE square root and division, no fused
// multiply-add); FP32 with the hardware reciprocal square root.
template <typename R, int DIM>
__device__ __forceinline__ void jump_sphere(R* x, R r, R z2, const R* z);
template <>
__device__ __forceinline__ void jump_sphere<double, 1>(double* x, double r, double z2, const double* z) {
#pragma clang fp contract(off)
  const double zn = sqrt(z2);
  x[0] = x[0] + r * (z[0] / zn);
}
template <>
__device__ __forceinline__ void jump_sphere<double, 2>(double* x, double r, double z2, const double* z) {
#pragma clang fp contract(off)
  const double zn = sqrt(z2);
  for (int k = 0; k < 2; ++k) x[k] = x[k] + r * (z[k] / zn);
}
template <>
__device__ __forceinline__ void jump_sphere<double, 3>(double* x, double r, double z2, const double* z) {
#pragma clang fp contract(off)
  const double zn = sqrt(z2);
  for (int k = 0; k < 3; ++k) x[k] = x[k] + r * (z[k] / zn);
}
template <int DIM>
__device__ __forceinline__ void jump_sphere_f(float* x, float r, float z2, const float* z) {
  const float s = r * __builtin_amdgcn_rsqf(z2);
#pragma unroll
  for (int k = 0; k < DIM; ++k) x[k] = x[k] + s * z[k];
}
template <>
__device__ __forceinline__ void jump_sphere<float, 1>(float* x, float r, float z2, const float* z) {
  jump_sphere_f<1>(x, r, z2, z);
}
template <>
__device__ __forceinline__ void jump_sphere<float, 2>(float* x, float r, float z2, const float* z) {
  jump_sphere_f<2>(x, r, z2, z);
}
template <>
__device__ __forceinline__ void jump_sphere<float, 3>(float* x, float r, float z2, const float* z) {
  jump_sphere_f<3>(x, r, z2, z);
}

// Nearest boundary point.  Outside a box: clamp; inside a box (censored path):
// the nearest face; ball: c + R (x - c)/|x - c| (c + R e_0 at the centre).
template <typename R, int DIM>
__device__ __forceinline__ void project(const Dom<R>& D, const R* x, R* out) {
#pragma unroll
  for (int k = 0; k < 3; ++k) out[k] = (k < DIM) ? x[k] : (R)0;
  if (D.kind == DOM_BOX) {
    if (!inside<R, DIM>(D, x)) {
#pragma unroll
      for (int k = 0; k < DIM; ++k) out[k] = fmin(fmax(x[k], D.lo[k]), D.hi[k]);
    } else {
      int best = 0;
      R bestd = (R)1e30, target = (R)0;
#pragma unroll
      for (int k = 0; k < DIM; ++k) {
        const R dl = x[k] - D.lo[k], dh = D.hi[k] - x[k];
        if (dl < bestd) { bestd = dl; best = k; target = D.lo[k]; }
        if (dh < bestd) { bestd = dh; best = k; target = D.hi[k]; }
      }
#pragma unroll
      for (int k = 0; k < DIM; ++k) if (k == best) out[k] = target;
    }
  } else {
    R r2 = (R)0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      const R d = x[k] - D.ctr[k];
      r2 += d * d;
    }
    const R r = sqrt(r2);
    if (r == (R)0) {
#pragma unroll
      for (int k = 0; k < DIM; ++k) out[k] = D.ctr[k] + (k == 0 ? D.rad : (R)0);
    } else {
      const R s = D.rad / r;
#pragma unroll
      for (int k = 0; k < DIM; ++k) out[k] = D.ctr[k] + s * (x[k] - D.ctr[k]);
    }
  }
}

// ---------------------------------------------------------------------------
// Wavefront reductions (64 lanes) with butterfly shuffles.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
__device__ __forceinline__ int64_t wave_sum(int64_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Chan et al. merge of Welford triples (n, mean, m2), written without
// branches (an empty side has n = 0 and mean = 0, which the formulas absorb:
// f = 0 keeps the left triple, f = 1 with n = 0 returns the right one).
__device__ __forceinline__ void chan_merge(double& n, double& mean, double& m2, double nb, double meanb,
                                           double m2b) {
  const double nn = n + nb;
  const double d = meanb - mean;
  const double f = nb / (nn > 0.0 ? nn : 1.0);
  mean = mean + d * f;
  m2 = m2 + m2b + d * d * n * f;
  n = nn;
}

// Butterfly merge; both partners merge (lower lane, upper lane) in that order,
// so every lane ends with the same bits.  Operand order is picked with
// selects, not branches, so the reduction adds no divergent control flow.
__device__ __forceinline__ void wave_welford(double& n, double& mean, double& m2) {
  const int lane = (int)(threadIdx.x & (kWave - 1));
#pragma unroll
  for (int o = 1; o <= 32; o <<= 1) {
    const double nb = __shfl_xor(n, o, kWave);
    const double mb = __shfl_xor(mean, o, kWave);
    const double qb = __shfl_xor(m2, o, kWave);
    const bool up = (lane & o) != 0;
    double an = up ? nb : n, am = up ? mb : mean, aq = up ? qb : m2;
    const double bn = up ? n : nb, bm = up ? mean : mb, bq = up ? m2 : qb;
    chan_merge(an, am, aq, bn, bm, bq);
    n = an;
    mean = am;
    m2 = aq;
  }
}

// Pops the next work-item index for the whole wavefront (call with all lanes
// active).  readfirstlane puts the index in a scalar register, so the
// compiler sees it as wave-uniform and the caller's "queue empty" exit is a
// uniform branch; a per-lane copy (e.g. a shuffle) makes that exit look
// divergent and can leave lanes without a fresh index.
// The atomic is issued by every lane (increment 1 from lane 0, 0 from the
// rest) rather than under `if (lane == 0)`: a lane-divergent branch here, ahead
// of the loop exit that tests the popped index, has been compiled into a
// nested loop whose exit mask was the lane-0 mask, sending lanes 1..63 back
// through the body with a stale index (a wave that never finishes).
__device__ __forceinline__ uint32_t pop_item(uint32_t* qhead) {
  const uint32_t inc = (threadIdx.x & (kWave - 1)) == 0 ? 1u : 0u;
  const uint32_t v = atomicAdd(qhead, inc);
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }
__device__ __forceinline__ int lane_rank(uint64_t mask) {
  // number of set bits of `mask` below this lane
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

}  // namespace pdd
