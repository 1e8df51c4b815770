// Launch schedules of the persistent kernels (paths or trees per work item,
// persistent grid per compute unit, step groups between lane refills).
//
// A call takes, for each knob, the caller's option when it is set, else the
// device's tuned entry for (kernel, dimension, precision), else the built-in
// default below.  Tuned entries come from pdd_set_schedule (the measured
// search in paper_1705_03666_amd/autotune.py calls it) and are kept per
// device kind (architecture and compute-unit count) in a text file, one entry
// per line, that the library reads on its first call and pdd_save_schedules
// writes: $PDD_SCHEDULE_FILE, or ~/.cache/pdd/schedules.txt.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>

#include <sys/stat.h>
#include <unistd.h>

#include "pdd_tuning.hpp"

namespace pdd {

namespace {

struct Entry {
  int32_t chunk, blocks, refill;
};

using Key = std::tuple<std::string, int, int, int>;  // device kind, kernel, dim, precision

std::mutex g_mu;
std::map<Key, Entry> g_table;
bool g_loaded = false;
std::string g_tags[64];

std::string default_path() {
  if (const char* p = std::getenv("PDD_SCHEDULE_FILE")) return p;
  const char* home = std::getenv("HOME");
  return std::string(home ? home : ".") + "/.cache/pdd/schedules.txt";
}

// Architecture and compute-unit count of the current device.
std::string device_tag() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return "unknown";
  if (g_tags[dev].empty()) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
    std::string arch(p.gcnArchName);
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch.resize(colon);
    g_tags[dev] = arch + "/" + std::to_string(p.multiProcessorCount);
  }
  return g_tags[dev];
}

// mkdir -p: every prefix of `dir` that ends before a '/' (and dir itself).
void make_dirs(const std::string& dir) {
  for (size_t i = 1; i <= dir.size(); ++i)
    if (i == dir.size() || dir[i] == '/') (void)::mkdir(dir.substr(0, i).c_str(), 0755);
}

bool valid(const Entry& e) {
  return e.chunk >= 1 && e.chunk <= (1 << 30) && e.blocks >= 1 && e.blocks <= 64 && e.refill >= 1 && e.refill <= 64;
}

int load_locked(const std::string& path) {
  std::ifstream in(path);
  if (!in) return -1;
  int n = 0;
  std::string line;
  while (std::getline(in, line)) {
    if (line.empty() || line[0] == '#') continue;
    std::istringstream ls(line);
    std::string tag;
    int kernel, dim, prec;
    Entry e;
    if (!(ls >> tag >> kernel >> dim >> prec >> e.chunk >> e.blocks >> e.refill)) continue;
    if (!valid(e)) continue;
    g_table[Key(tag, kernel, dim, prec)] = e;
    ++n;
  }
  return n;
}

void ensure_loaded_locked() {
  if (!g_loaded) {
    g_loaded = true;
    (void)load_locked(default_path());
  }
}

bool lookup(int kernel, int dim, int precision, Entry* out) {
  std::lock_guard<std::mutex> lock(g_mu);
  ensure_loaded_locked();
  auto it = g_table.find(Key(device_tag(), kernel, dim, precision));
  if (it == g_table.end()) return false;
  *out = it->second;
  return true;
}

// Built-in defaults, measured on MI355X: the 3-D C5 walk (forward and
// adjoint alike) for the linear kernels; C4 / C7 (k_branch) and C6
// (k_branch_bvp), 1024 points x 1e5 trees, for branching: four blocks per
// CU (the FP32 branching kernels are built for four waves per SIMD, and
// their LDS stacks allow four blocks), items of 16384 trees for k_branch
// (C4: 3.36 ms against 3.60 with 8192 and 4.77 with 32768; 2 blocks and
// 2048-tree items took 2.0x) and of 8192 trees for k_branch_bvp, whose trees
// are long enough that the last items of a launch decide its end (C6: 233.5
// ms against 238.1 with 4096).
Entry defaults(int kernel, bool fp32, int dim) {
  (void)dim;
  if (kernel == PDD_KERNEL_BRANCH) return Entry{16384, fp32 ? 4 : 2, 1};
  if (kernel == PDD_KERNEL_BRANCH_BVP) return Entry{8192, fp32 ? 4 : 2, 1};
  // the adjoint / value+Jacobian walk: the autotuner's choice on C5 (items of
  // 32768 paths, 0.3-1% ahead of 16384)
  if (kernel == PDD_KERNEL_WALK_ADJOINT && fp32) return Entry{32768, 8, 3};
  // the heterogeneous batch: items of 4096 paths, 6 blocks per CU (C3, Euler:
  // 27.3 ms against 28.7 with 2048 and 27.8 with 8192), refills every 6 step
  // groups for Euler (27.9 ms with 4, 29.3 with 2), every 2 for walk on
  // spheres, whose paths are short (3.83 ms against 4.04 with 4, 4.47 with 6)
  if (kernel == PDD_KERNEL_WALK_BATCH) return Entry{4096, fp32 ? 6 : 4, 6};
  if (kernel == PDD_KERNEL_WOS_BATCH) return Entry{4096, fp32 ? 6 : 4, 2};
  return Entry{16384, fp32 ? 8 : 4, 3};
}

}  // namespace

Tuning choose_schedule(int kernel, int dim, int precision, const pdd_options& o, int n_cus, int64_t total_work) {
  const bool fp32 = precision == PDD_FP32_STEP;
  Entry e = defaults(kernel, fp32, dim);
  Entry tuned;
  if (lookup(kernel, dim, precision, &tuned)) e = tuned;
  Tuning t;
  t.chunk_paths = e.chunk;
  t.blocks_per_cu = e.blocks;
  t.refill_groups = e.refill;
  if (o.blocks_per_cu > 0) t.blocks_per_cu = o.blocks_per_cu;
  if (o.refill_groups > 0) t.refill_groups = o.refill_groups;
  if (o.chunk_paths > 0) {
    t.chunk_paths = o.chunk_paths;
  } else {
    // a call too small for the item size: halve it (down to 1024 paths)
    // until every resident wavefront gets several items (the walks: four;
    // branching: one, its items being longer)
    const int64_t waves = (int64_t)t.blocks_per_cu * std::max(1, n_cus) * 4;
    const int64_t per_wave = (kernel == PDD_KERNEL_BRANCH || kernel == PDD_KERNEL_BRANCH_BVP) ? 1 : 4;
    while (t.chunk_paths > 1024 && total_work / t.chunk_paths < per_wave * waves) t.chunk_paths /= 2;
  }
  t.chunk_paths = std::max(1, t.chunk_paths);
  return t;
}

bool schedule_kind_valid(int kernel, int dim, int precision) {
  return kernel >= PDD_KERNEL_WALK && kernel <= PDD_KERNEL_BRANCH_BVP && dim >= 0 && dim <= 3 &&
         (precision == PDD_FP64 || precision == PDD_FP32_STEP);
}

int set_schedule(int kernel, int dim, int precision, const pdd_launch_schedule* s) {
  std::lock_guard<std::mutex> lock(g_mu);
  ensure_loaded_locked();
  const Key k(device_tag(), kernel, dim, precision);
  if (s == nullptr) {
    g_table.erase(k);
    return 0;
  }
  const Entry e{s->chunk_paths, s->blocks_per_cu, s->refill_groups};
  if (!valid(e)) return -1;
  g_table[k] = e;
  return 0;
}

int get_schedule(int kernel, int dim, int precision, pdd_launch_schedule* out, int32_t* tuned) {
  Entry e;
  const bool have = lookup(kernel, dim, precision, &e);
  if (!have) e = defaults(kernel, precision == PDD_FP32_STEP, dim);
  if (out) {
    out->chunk_paths = e.chunk;
    out->blocks_per_cu = e.blocks;
    out->refill_groups = e.refill;
    out->pad = 0;
  }
  if (tuned) *tuned = have ? 1 : 0;
  return 0;
}

int save_schedules(const char* path) {
  std::lock_guard<std::mutex> lock(g_mu);
  ensure_loaded_locked();
  const std::string p = path ? std::string(path) : default_path();
  const size_t slash = p.find_last_of('/');
  if (slash != std::string::npos && slash > 0) make_dirs(p.substr(0, slash));
  const std::string tmp = p + ".tmp" + std::to_string((long)::getpid());
  {
    std::ofstream out(tmp);
    if (!out) return -1;
    out << "# pdd launch schedules: device kernel dim precision chunk_paths blocks_per_cu refill_groups\n";
    for (const auto& kv : g_table) {
      const Key& k = kv.first;
      const Entry& e = kv.second;
      out << std::get<0>(k) << ' ' << std::get<1>(k) << ' ' << std::get<2>(k) << ' ' << std::get<3>(k) << ' '
          << e.chunk << ' ' << e.blocks << ' ' << e.refill << '\n';
    }
    if (!out) return -1;
  }
  if (std::rename(tmp.c_str(), p.c_str()) != 0) {
    std::remove(tmp.c_str());
    return -1;
  }
  return 0;
}

int load_schedules(const char* path) {
  std::lock_guard<std::mutex> lock(g_mu);
  g_loaded = true;
  return load_locked(path ? std::string(path) : default_path());
}

}  // namespace pdd
