// Host-only check of the problem-specialised kernels: generates their sources
// for a few problem structures with the library's own generators and
// compiles them with the library's runtime-compilation step for the target
// given as argv[1] (default gfx950), without loading them, so no GPU is
// needed.  Prints one line per kernel; exit status 0 when every kernel
// compiled and every non-literal structure was refused.
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "pdd_spec.hpp"

using namespace pdd;

namespace {

DevFactor fac(int fn, int dim, int power, double a, double b) {
  DevFactor f{};
  f.fn = fn;
  f.dim = dim;
  f.power = power;
  f.ad = a;
  f.bd = b;
  f.af = (float)a;
  f.bf = (float)b;
  return f;
}

DevFun fun(int n_terms, int n_factors, int fac_off, int coef_off, int poly_deg = -1, int poly_off = 0) {
  DevFun F{};
  F.n_terms = n_terms;
  F.n_factors = n_factors;
  F.fac_off = fac_off;
  F.coef_off = coef_off;
  F.poly_deg = poly_deg;
  F.poly_off = poly_off;
  return F;
}

int failures = 0;

// `policy` is a generated policy struct; `branch` selects the kernel header
// it is compiled with (branching or walk), as the library's loaders do.
void check(const std::string& what, const std::string& policy, bool branch, const std::string& name,
           const std::string& arch) {
  if (policy.empty()) {
    std::printf("FAIL %s: no source generated\n", what.c_str());
    ++failures;
    return;
  }
  const std::string src = branch ? spec_branch_source(policy) : spec_walk_source(policy);
  std::string code, lowered, err;
  if (!spec_compile(src, name, arch, &code, &lowered, &err)) {
    std::printf("FAIL %s (%s): %s\n", what.c_str(), name.c_str(), err.c_str());
    ++failures;
    return;
  }
  std::printf("ok %s: %s, %zu bytes, %s\n", what.c_str(), name.c_str(), code.size(), lowered.c_str());
}

}  // namespace

int main(int argc, char** argv) {
  const std::string arch = argc > 1 ? argv[1] : "gfx950";

  // psi = c0 + c1 tanh(x0) (a padded constant term), free branching, FP32, 3-D
  std::vector<DevFactor> f1 = {fac(FN_POW, 0, 0, 1.0, 0.0), fac(FN_TANH, 0, 1, 1.0, 0.0)};
  const DevFun psi1 = fun(2, 1, 0, 0);
  check("free FP32 3-D", spec_psi_source(psi1, nullptr, f1), true, spec_branch_name(true, 3, RNG_QUAD24, false),
        arch);

  // psi with terms and a dense polynomial part, FP64, 1-D, both layouts
  std::vector<DevFactor> f2 = {fac(FN_EXP, 0, 2, -0.5, 0.25), fac(FN_COS, 0, 1, 3.0, 0.0)};
  const DevFun psi2 = fun(1, 2, 0, 0, 3, 1);
  for (int layout : {RNG_PAIR52, RNG_QUAD24})
    check("free FP64 1-D", spec_psi_source(psi2, nullptr, f2), true, spec_branch_name(false, 1, layout, false),
          arch);

  // boundary: psi with three terms, g with six terms of two factors, one of
  // them in the time argument (coordinate dim), FP32, 1-D
  std::vector<DevFactor> f3 = {fac(FN_POW, 0, 0, 1, 0), fac(FN_TANH, 0, 1, 0.2, 0), fac(FN_TANH, 0, 2, 0.2, 0)};
  for (int b = 0; b < 2; ++b) {
    const DevFactor w = fac(FN_POW, 0, 1, b ? 0.1 : -0.1, 0.5);
    f3.push_back(w);
    f3.push_back(fac(FN_POW, 0, 0, 1, 0));
    f3.push_back(w);
    f3.push_back(fac(FN_TANH, 1, 1, -5.0 / 12.0, b ? 1.0 : -1.0));
    f3.push_back(w);
    f3.push_back(fac(FN_TANH, 1, 2, -5.0 / 12.0, b ? 1.0 : -1.0));
  }
  const DevFun psi3 = fun(3, 1, 0, 0), g3 = fun(6, 2, 3, 3);
  check("boundary FP32 1-D", spec_psi_source(psi3, &g3, f3), true, spec_branch_name(true, 1, RNG_QUAD24, true),
        arch);

  // boundary, FP64, 3-D: g with a polynomial part and a sine of the time argument
  std::vector<DevFactor> f4 = {fac(FN_COS, 1, 1, 1.0, 0.0), fac(FN_SIN, 3, 1, 1.3, 0.0)};
  const DevFun psi4 = fun(1, 1, 0, 0), g4 = fun(1, 1, 1, 1, 2, 2);
  check("boundary FP64 3-D", spec_psi_source(psi4, &g4, f4), true, spec_branch_name(false, 3, RNG_PAIR52, true),
        arch);

  // the walk: b, c and f with generic terms, 2-D forward and 3-D adjoint
  LinearParams P{};
  std::vector<DevFactor> f5 = {fac(FN_SIN, 1, 1, 3.14159, 0), fac(FN_COS, 0, 1, 3.14159, 0),
                               fac(FN_POW, 0, 2, 1, 0),     fac(FN_EXP, 1, 1, 1, 0),
                               fac(FN_COS, 0, 1, 1, 0)};
  P.b[0] = fun(1, 1, 0, 0);
  P.b[1] = fun(1, 1, 1, 1);
  P.b[2] = fun(0, 0, 0, 0);
  P.c = fun(1, 1, 2, 2);
  P.f = fun(1, 2, 3, 3);
  P.g = fun(0, 0, 0, 0);
  check("walk FP32 2-D", spec_terms_source(P, f5), false, spec_walk_name(true, 2, -1, RNG_QUAD24, false), arch);
  check("walk adjoint FP32 3-D", spec_terms_source(P, f5), false, spec_walk_name(true, 3, -1, RNG_QUAD24, true),
        arch);

  // a scale that cannot be written as a literal: no source, so the library
  // runs the table-driven kernel
  std::vector<DevFactor> f6 = {fac(FN_TANH, 0, 1, std::nan(""), 0.0)};
  const DevFun psi6 = fun(1, 1, 0, 0);
  if (!spec_psi_source(psi6, nullptr, f6).empty()) {
    std::printf("FAIL non-finite scale: a source was generated\n");
    ++failures;
  } else {
    std::printf("ok non-finite scale refused\n");
  }
  return failures == 0 ? 0 : 1;
}
