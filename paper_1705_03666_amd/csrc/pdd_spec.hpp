// Problem-specialised walk and branching kernels (host side).
//
// A problem whose b, c or f carry generic terms (products of exp, sin, cos,
// tanh and powers of affine functions of one coordinate) pays, in the
// precompiled kernels, for reading and dispatching on every factor record at
// every step.  Instead the library writes the factor structure of that
// problem (functions, coordinates, scales, shifts, powers) into C++ source as
// constants, compiles k_walk with it at run time for the device in use, and
// launches the result.  Coefficients stay run-time data, so one compiled
// kernel serves every coefficient value: each thread copies the term
// coefficients of b, c and f from the staged table into VGPRs once per launch
// (a product whose operands are all VGPRs can issue in the same cycle as
// another wavefront's instruction that reads a scalar register), while g's
// stay in the table.  The specialised kernel evaluates the same products in
// the same order as the table-driven one.
//
// The branching kernels get the same treatment for psi (at leaves and output
// times) and g (at boundary stops): a generated policy struct with their
// factor structure written in replaces the table walk; coefficients are read
// from the staged table as in the table-driven kernels, and the results are
// the same bits.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "pdd_internal.hpp"

namespace pdd {

// Source of the term policy (struct pdd_spec::SpecTerms) for the functions
// described by P.b, P.c, P.f, P.g and the factor records `fac`; empty when a
// value cannot be written as a literal (non-finite scale or shift).
std::string spec_terms_source(const LinearParams& P, const std::vector<DevFactor>& fac);

// Loads (compiling on first use, per device) the k_walk instantiation
// <R, DIM, DFC, LAYOUT, TERMS = true, ADJ, WOS = false, SpecTerms>.  Returns
// false with a message in *err when the runtime compiler or the module load
// fails.  Compiled code objects are kept in memory for the life of the
// process and, when the directory is writable, in $PDD_JIT_CACHE (default
// ~/.cache/pdd_jit).
bool spec_walk_kernel(const std::string& terms_src, bool fp32, int dim, int dfc, int layout, bool adjoint,
                      hipFunction_t* fn, std::string* err);

// Source of the psi / g policy (struct pdd_spec::SpecPsi) of the branching
// kernels for psi (and, with a boundary, g: coordinates 0..dim-1 and the time
// argument as coordinate dim) described by the factor records `fac`; empty
// when a value cannot be written as a literal.
std::string spec_psi_source(const DevFun& psi, const DevFun* g, const std::vector<DevFactor>& fac);

// Loads (compiling on first use, per device) k_branch<R, DIM, LAYOUT,
// SpecPsi>, or k_branch_bvp with `boundary`; caches and errors as for
// spec_walk_kernel.
bool spec_branch_kernel(const std::string& psi_src, bool fp32, int dim, int layout, bool boundary,
                        hipFunction_t* fn, std::string* err);

// The pieces of the two loaders above, for checks that compile without
// loading (no GPU needed): the instantiation names and full sources of the
// specialised kernels, and the runtime compilation itself (code object and
// lowered kernel name for the target `arch`, e.g. "gfx950"; false with the
// compiler log in *err on failure).
std::string spec_walk_name(bool fp32, int dim, int dfc, int layout, bool adjoint);
std::string spec_walk_source(const std::string& terms_src);
std::string spec_branch_name(bool fp32, int dim, int layout, bool boundary);
std::string spec_branch_source(const std::string& psi_src);
bool spec_compile(const std::string& src, const std::string& name, const std::string& arch, std::string* code,
                  std::string* lowered, std::string* err);

}  // namespace pdd
