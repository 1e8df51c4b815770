// Library-lifetime device memory (noalloc.hip) and the host-layer entry the
// allocation-free interface call runs through (capi.cpp).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include <string>

#include "pdd.h"

namespace pdd {

constexpr int kMaxDevices = 64;
// Scratch of pdd_mc_interface_noalloc: its staged tables, node copy, work
// queue and per-item partials must fit (C5-sized forward calls, 4096 nodes x
// 1e5 paths, take about 4 MB).
constexpr size_t kFixedScratchBytes = (size_t)16 << 20;

// The current device's addresses of the fixed scratch area and of the two
// warning counters (looked up once per device, on first use).
hipError_t fixed_symbols(void** scratch, unsigned long long** counters);

// Sets the thread's last-error message and returns `s`.
pdd_status set_error(pdd_status s, const std::string& msg);

// pdd_mc_interface with every device buffer carved out of `area` (bytes
// long): nothing is allocated; the runtime-compiled specialised kernels are
// not used (loading one maps memory).
pdd_status run_linear_fixed(const pdd_linear_problem* problem, const double* nodes_dev, int64_t n_nodes,
                            const int64_t* paths_host, double dt, uint64_t seed, const pdd_options* options,
                            pdd_node_stat* out_dev, void* area, size_t bytes, void* hip_stream);

}  // namespace pdd
