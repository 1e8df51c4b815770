// Library-lifetime device memory: the fixed scratch area of the
// allocation-free entry point pdd_mc_interface_noalloc, and the warning
// counters (censored paths, redrawn trees) that every entry point adds to.
//
// Both are file-scope device arrays, so no call maps memory for them.  Host
// code never uses their names as addresses: on first use on a device (with
// that device current) hipGetSymbolAddress gives each array's address on
// that device, which is kept per device and passed to the kernels.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "pdd.h"
#include "pdd_fixed.hpp"

namespace pdd {

static __device__ __align__(256) unsigned char scratch[kFixedScratchBytes];
static __device__ __align__(16) unsigned long long warn_counters[2];

namespace {

struct DeviceSymbols {
  void* scratch = nullptr;
  unsigned long long* counters = nullptr;
};

std::mutex g_sym_mu;
DeviceSymbols g_syms[kMaxDevices];

}  // namespace

hipError_t fixed_symbols(void** scratch_out, unsigned long long** counters_out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_sym_mu);
  DeviceSymbols& s = g_syms[dev];
  if (s.scratch == nullptr) {
    void* p = nullptr;
    void* c = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    e = hipGetSymbolAddress(&c, HIP_SYMBOL(warn_counters));
    if (e != hipSuccess) return e;
    if (p == nullptr || c == nullptr) return hipErrorInvalidSymbol;
    s.scratch = p;
    s.counters = (unsigned long long*)c;
  }
  if (scratch_out) *scratch_out = s.scratch;
  if (counters_out) *counters_out = s.counters;
  return hipSuccess;
}

}  // namespace pdd

extern "C" pdd_status pdd_mc_interface_noalloc(const pdd_linear_problem* problem, const double* nodes_dev,
                                                int64_t n_nodes, const int64_t* paths_host, double dt,
                                                uint64_t seed, const pdd_options* options, pdd_node_stat* out_dev,
                                                void* hip_stream) {
  void* area = nullptr;
  const hipError_t e = pdd::fixed_symbols(&area, nullptr);
  if (e != hipSuccess)
    return pdd::set_error(PDD_ERR_HIP, std::string("scratch symbol address: ") + hipGetErrorString(e));
  return pdd::run_linear_fixed(problem, nodes_dev, n_nodes, paths_host, dt, seed, options, out_dev, area,
                               pdd::kFixedScratchBytes, hip_stream);
}
