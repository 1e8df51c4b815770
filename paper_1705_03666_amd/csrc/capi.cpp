// Host layer of the C ABI declared in include/pdd.h: argument validation,
// staging of coefficient tables, work-item construction (longest first),
// launch of the HIP kernels on the caller's stream, cached hipGraph launch
// plans, and warning counters.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "pdd.h"
#include "pdd_internal.hpp"
#include "pdd_kernels.hpp"
#include "pdd_spec.hpp"
#include "pdd_fixed.hpp"
#include "pdd_tuning.hpp"

using namespace pdd;

namespace {

thread_local std::string g_last_error;

pdd_status fail(pdd_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

#define PDD_HIP(call)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess) return fail(PDD_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// ----------------------------------------------------------------------------- call arenas
// Every call takes its device buffers (tables, work queue, per-item
// statistics, branching stack) as one stream-ordered arena.  They come from a
// memory pool of the library's own, one per device, that keeps up to
// kPoolKeep bytes mapped after a free, so a repeated call maps no new memory
// (the largest arena at the workloads here, the 1024-point branching spill
// area, is about 0.8 GB); beyond that the pool returns memory at the next
// synchronisation.  pdd_release_workspace() returns all of it.  The
// process's default pool is left as it is.
constexpr uint64_t kPoolKeep = 2ull << 30;
std::mutex g_pool_mu;
std::vector<hipMemPool_t> g_pools;  // by device ordinal

hipError_t arena_alloc(void** p, size_t bytes, hipStream_t st) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  hipMemPool_t pool = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_pool_mu);
    if ((int)g_pools.size() <= dev) g_pools.resize(dev + 1, nullptr);
    if (g_pools[dev] == nullptr) {
      hipMemPoolProps pr;
      std::memset(&pr, 0, sizeof(pr));
      pr.allocType = hipMemAllocationTypePinned;
      pr.location.type = hipMemLocationTypeDevice;
      pr.location.id = dev;
      hipMemPool_t np = nullptr;
      e = hipMemPoolCreate(&np, &pr);
      if (e != hipSuccess) return e;
      uint64_t keep = kPoolKeep;
      e = hipMemPoolSetAttribute(np, hipMemPoolAttrReleaseThreshold, &keep);
      if (e != hipSuccess) {
        (void)hipMemPoolDestroy(np);
        return e;
      }
      g_pools[dev] = np;
    }
    pool = g_pools[dev];
  }
  return hipMallocFromPoolAsync(p, bytes, pool, st);
}

// The call arena of a (device, stream): kept from one call to the next and
// grown when a call needs more, so a call frees nothing (a stream-ordered
// free here waited for the work queued before it: about 3 ms per C4 call,
// which made every call block the host).  Calls on one stream run in order,
// so a call's uploads into the arena cannot overtake the previous call's
// kernels; the lease holds the arena's lock while a call enqueues, so two host
// threads cannot interleave their uploads and launches on one stream.  An
// event recorded after each use orders the next one even if the stream handle
// is reused by a new stream.  pdd_release_workspace() returns the memory.
struct StreamArena {
  int dev = 0;
  hipStream_t st = nullptr;
  void* p = nullptr;
  size_t bytes = 0;
  hipEvent_t last = nullptr;
  std::mutex mu;
};
std::mutex g_sa_mu;
std::vector<std::unique_ptr<StreamArena>> g_stream_arenas;

struct ArenaLease {
  StreamArena* a = nullptr;
  std::unique_lock<std::mutex> lk;
  hipStream_t st = nullptr;
  // marks the end of this call's use (after its last launch)
  hipError_t done() { return a != nullptr ? hipEventRecord(a->last, st) : hipSuccess; }
};

hipError_t lease_arena(size_t bytes, hipStream_t st, ArenaLease* L, void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  StreamArena* a = nullptr;
  {
    std::lock_guard<std::mutex> g(g_sa_mu);
    for (auto& x : g_stream_arenas)
      if (x->dev == dev && x->st == st) {
        a = x.get();
        break;
      }
    if (a == nullptr) {
      g_stream_arenas.emplace_back(new StreamArena());
      a = g_stream_arenas.back().get();
      a->dev = dev;
      a->st = st;
    }
  }
  L->lk = std::unique_lock<std::mutex>(a->mu);
  L->a = a;
  L->st = st;
  if (a->last == nullptr) {
    if ((e = hipEventCreateWithFlags(&a->last, hipEventDisableTiming)) != hipSuccess) return e;
  } else if ((e = hipStreamWaitEvent(st, a->last, 0)) != hipSuccess) {
    return e;
  }
  if (a->bytes < bytes) {
    if (a->p != nullptr && (e = hipFreeAsync(a->p, st)) != hipSuccess) return e;
    a->p = nullptr;
    a->bytes = 0;
    const size_t nb = (bytes + ((size_t)2 << 20) - 1) & ~(((size_t)2 << 20) - 1);   // 2 MiB granules
    if ((e = arena_alloc(&a->p, nb, st)) != hipSuccess) return e;
    a->bytes = nb;
  }
  *out = a->p;
  return hipSuccess;
}

// Returns every call arena (after a device synchronisation; no call may run).
hipError_t release_stream_arenas() {
  std::lock_guard<std::mutex> g(g_sa_mu);
  for (auto& x : g_stream_arenas) {
    std::lock_guard<std::mutex> lk(x->mu);
    if (x->p != nullptr) {
      hipError_t e = hipFreeAsync(x->p, nullptr);
      if (e != hipSuccess) return e;
    }
    if (x->last != nullptr) (void)hipEventDestroy(x->last);
  }
  g_stream_arenas.clear();
  return hipDeviceSynchronize();
}

// Unmaps every page the library pools hold (call after a device synchronisation).
hipError_t trim_pools() {
  std::lock_guard<std::mutex> lock(g_pool_mu);
  for (hipMemPool_t p : g_pools)
    if (p != nullptr) {
      hipError_t e = hipMemPoolTrimTo(p, 0);
      if (e != hipSuccess) return e;
    }
  return hipSuccess;
}

// ----------------------------------------------------------------------------- monomials
int n_mono(int dim, int deg) {
  if (deg < 0) return 0;
  int r = 1;
  for (int i = 1; i <= dim; ++i) r = r * (deg + i) / i;
  return r;
}

std::vector<std::array<int, 3>> graded_lex(int dim, int deg) {
  std::vector<std::array<int, 3>> out;
  for (int k = 0; k <= deg; ++k) {
    if (dim == 1) {
      out.push_back({k, 0, 0});
    } else if (dim == 2) {
      for (int a = k; a >= 0; --a) out.push_back({a, k - a, 0});
    } else {
      for (int a = k; a >= 0; --a)
        for (int b = k - a; b >= 0; --b) out.push_back({a, b, k - a - b});
    }
  }
  return out;
}

// nested order (a outer, b middle, c inner) -> graded-lex index
std::vector<int32_t> nested_to_graded(int dim, int deg) {
  auto gl = graded_lex(dim, deg);
  std::vector<int32_t> out;
  for (int a = 0; a <= deg; ++a)
    for (int b = 0; b <= (dim >= 2 ? deg - a : 0); ++b)
      for (int c = 0; c <= (dim >= 3 ? deg - a - b : 0); ++c) {
        std::array<int, 3> e = {a, b, c};
        for (size_t i = 0; i < gl.size(); ++i)
          if (gl[i] == e) { out.push_back((int32_t)i); break; }
      }
  return out;
}

// ----------------------------------------------------------------------------- validation
pdd_status check_fun(const pdd_fun& F, int dim, const char* name, int max_terms, int max_deg) {
  const std::string n(name);
  if (F.n_terms < 0 || F.n_terms > max_terms)
    return fail(F.n_terms < 0 ? PDD_ERR_INVALID_ARG : PDD_ERR_UNSUPPORTED,
                n + ": n_terms out of range (max " + std::to_string(max_terms) + ")");
  if (F.n_terms > 0) {
    if (F.n_factors < 0 || F.n_factors > kMaxFactors) return fail(PDD_ERR_UNSUPPORTED, n + ": n_factors must be 0..4");
    if (F.n_factors > 0 && F.factors == nullptr) return fail(PDD_ERR_INVALID_ARG, n + ": factors is NULL");
    if (F.coef == nullptr) return fail(PDD_ERR_INVALID_ARG, n + ": coef is NULL");
    for (int i = 0; i < F.n_terms * F.n_factors; ++i) {
      const pdd_factor& fa = F.factors[i];
      if (fa.fn < PDD_FN_POW || fa.fn > PDD_FN_TANH) return fail(PDD_ERR_INVALID_ARG, n + ": unknown factor kind");
      if (fa.dim < 0 || fa.dim >= dim) return fail(PDD_ERR_INVALID_ARG, n + ": factor dimension out of range");
      if (fa.power < 0 || fa.power > 16) return fail(PDD_ERR_INVALID_ARG, n + ": factor power must be 0..16");
      if (!std::isfinite(fa.a) || !std::isfinite(fa.b)) return fail(PDD_ERR_INVALID_ARG, n + ": non-finite factor");
    }
  }
  if (F.poly_degree < -1) return fail(PDD_ERR_INVALID_ARG, n + ": poly_degree < -1");
  if (F.poly_degree > max_deg)
    return fail(PDD_ERR_UNSUPPORTED, n + ": poly_degree above " + std::to_string(max_deg));
  if (F.poly_degree >= 0 && F.poly == nullptr) return fail(PDD_ERR_INVALID_ARG, n + ": poly is NULL");
  return PDD_OK;
}

bool is_zero_fun(const pdd_fun& F) { return F.n_terms == 0 && F.poly_degree < 0; }

pdd_status check_device_ptr(const void* p, const char* name) {
  if (p == nullptr) return fail(PDD_ERR_INVALID_ARG, std::string(name) + " is NULL");
  hipPointerAttribute_t attr;
  hipError_t e = hipPointerGetAttributes(&attr, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(PDD_ERR_INVALID_ARG, std::string(name) + " is not device memory");
  }
  if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
    return fail(PDD_ERR_INVALID_ARG, std::string(name) + " is not device memory");
  return PDD_OK;
}

// ----------------------------------------------------------------------------- tables
// Where a staging job reads from: coefficient array `part` (0 = coef, 1 =
// poly, 2 = none: zero padding, 3 = node coordinates) of function `fun`
// (0..2 = b, 3 = c, 4 = f, 5 = g; -1 = not recorded).
struct JobSource {
  int fun, part;
  int prob;   // problem index within a batch call (0 otherwise)
};

struct Tables {
  std::vector<DevFactor> fac;
  std::vector<StageJob> jobs;
  std::vector<JobSource> src;
  std::vector<int32_t> perm;
  int ncoef = 0;
  int cur_prob = 0;   // problem the next functions belong to (batch calls)

  void job(const StageJob& j, int fun, int part) {
    jobs.push_back(j);
    src.push_back(JobSource{fun, part, cur_prob});
  }

  DevFun add(const pdd_fun& F, int dim, int pad_deg, bool nested, int fun = -1) {
    DevFun d{};
    d.n_terms = F.n_terms;
    d.n_factors = F.n_terms > 0 ? F.n_factors : 0;
    d.fac_off = (int)fac.size();
    for (int i = 0; i < F.n_terms * d.n_factors; ++i) {
      const pdd_factor& s = F.factors[i];
      DevFactor t{};
      t.fn = s.fn; t.dim = s.dim; t.power = s.power;
      t.ad = s.a; t.bd = s.b; t.af = (float)s.a; t.bf = (float)s.b;
      fac.push_back(t);
    }
    d.coef_off = ncoef;
    if (F.n_terms > 0) {
      job(StageJob{F.coef, nullptr, ncoef, F.n_terms, -1, 0}, fun, 0);
      ncoef += F.n_terms;
    }
    d.poly_deg = -1;
    d.n_mono = 0;
    d.poly_off = ncoef;
    if (F.poly_degree >= 0) {
      const int own = n_mono(dim, F.poly_degree);
      if (nested) {
        auto p = nested_to_graded(dim, F.poly_degree);
        const int poff = (int)perm.size();
        perm.insert(perm.end(), p.begin(), p.end());
        job(StageJob{F.poly, nullptr, ncoef, own, poff, 0}, fun, 1);
        d.poly_deg = F.poly_degree;
        d.n_mono = own;
        ncoef += own;
      } else {
        const int deg = std::max(pad_deg, F.poly_degree);
        const int tot = n_mono(dim, deg);
        job(StageJob{F.poly, nullptr, ncoef, own, -1, 0}, fun, 1);
        if (tot > own) job(StageJob{nullptr, nullptr, ncoef + own, tot - own, -1, 0}, fun, 2);
        d.poly_deg = deg;
        d.n_mono = tot;
        ncoef += tot;
      }
    }
    return d;
  }
};

// ----------------------------------------------------------------------------- device arena
// One allocation carved into aligned pieces.
struct Arena {
  std::vector<std::pair<size_t, size_t>> parts;  // offset, size
  size_t total = 0;
  size_t add(size_t bytes) {
    const size_t off = (total + 255) & ~(size_t)255;
    total = off + std::max<size_t>(bytes, 1);
    return off;
  }
};

int device_cus() {
  static int cus[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (dev < 0 || dev >= 64) return 256;
  if (cus[dev] == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
    cus[dev] = v;
  }
  return cus[dev];
}

// per-device warning counters (censored paths, redrawn trees): a device
// array of the library (zero when the library is loaded), never allocated
std::mutex g_mu;

pdd_status counters(unsigned long long** out) {
  int dev = 0;
  PDD_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(PDD_ERR_UNSUPPORTED, "device index above 63");
  PDD_HIP(fixed_symbols(nullptr, out));
  return PDD_OK;
}

// ----------------------------------------------------------------------------- plans
// Everything a call enqueues, with its device buffers.  `enqueue` issues only
// kernel launches (no memset, no copies), so it can be captured in a graph.
// The caller's per-call pointers (node coordinates and coefficient arrays,
// through the staging jobs; outputs and weights, through CallPtrs) are read
// from the call block at the start of the arena, which is uploaded before
// every launch: a graph plan is keyed on what shapes the launch, not on the
// caller's buffers.
struct Plan {
  int device = 0;
  void* arena = nullptr;
  bool owned = false;   // hipMalloc'd (graph plan) vs stream-ordered
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  hipEvent_t done = nullptr;   // recorded after every launch of a graph plan
  uint64_t last_use = 0;

  LinearParams lp{};
  BranchParams bp{};
  BranchBoundary bb{};
  bool branch = false;
  bool bvp = false;          // branching with a boundary: istat is [n_times][n_items]
  int n_times = 1;
  BranchBvpLaunch bvl{};
  bool plain = false;
  bool adjoint = false;
  WalkLaunch wl{};
  BranchLaunch bl{};
  std::vector<PlainLaunch> pl;
  bool batch = false;        // heterogeneous batch of linear problems
  WalkBatchLaunch wbl{};

  CallPtrs* d_call = nullptr;   // call block: CallPtrs, then the staging jobs
  StageJob* d_jobs = nullptr;
  int n_jobs = 0;
  std::vector<StageJob> jobs_host;   // graph plans: the staging jobs as captured,
  std::vector<JobSource> job_src;    // with where each one reads from
  double* d_nodes = nullptr;         // staged node coordinates
  int32_t* d_perm = nullptr;
  double* d_cd = nullptr;
  float* d_cf = nullptr;
  uint32_t* d_qhead = nullptr;
  ItemStat* d_istat = nullptr;
  int64_t* d_first = nullptr;
  int64_t n_nodes = 0;
  bool has_out = false;
  unsigned long long* ctr = nullptr;

  // adjoint reduction
  double* d_igrad = nullptr;
  int grad_stride = 0;
  int n_items = 0;
  int32_t* d_slot_node = nullptr;
  double* d_inv_n = nullptr;
  bool has_w = false;
  double* d_colsum = nullptr;
  int32_t* d_gmap = nullptr;
  struct Scatter { int col, count; bool gmap; int which; };
  std::vector<Scatter> scatters;
  // value+Jacobian mode
  bool has_jac = false;
  int64_t jac_ld = 0;
  int32_t* d_colmap = nullptr;
  int n_jcols = 0;

  hipError_t enqueue(hipStream_t st) const {
    hipError_t e;
    if ((e = launch_stage(d_jobs, n_jobs, d_perm, d_cd, d_cf, st)) != hipSuccess) return e;
    if (plain) {
      for (const auto& L : pl)
        if ((e = (L.adjoint ? launch_plain_adj(L, st) : launch_plain(L, st))) != hipSuccess) return e;
      if (!adjoint) return launch_finalize_nodes(d_istat, d_first, n_nodes, d_call, 0, ctr, st);
    } else {
      if ((e = launch_fill_u32(d_qhead, 1, 0u, st)) != hipSuccess) return e;
      if (bvp) {
        if ((e = launch_branch_bvp(bvl, st)) != hipSuccess) return e;
        for (int k = 0; k < n_times; ++k)
          if ((e = launch_finalize_nodes(d_istat + (size_t)k * n_items, d_first, n_nodes, d_call,
                                         (int64_t)k * n_nodes, k == 0 ? ctr : nullptr, st)) != hipSuccess)
            return e;
        return hipSuccess;
      } else if (branch) {
        if ((e = launch_branch(bl, st)) != hipSuccess) return e;
      } else if (batch) {
        if ((e = launch_walk_batch(wbl, st)) != hipSuccess) return e;
      } else {
        if ((e = launch_walk(wl, st)) != hipSuccess) return e;
      }
    }
    if (has_out)
      if ((e = launch_finalize_nodes(d_istat, d_first, n_nodes, d_call, 0, ctr, st)) != hipSuccess) return e;
    if (adjoint && has_w) {
      if ((e = launch_finalize_grad(d_igrad, grad_stride, grad_stride, n_items, d_slot_node, d_call, d_inv_n,
                                    d_colsum, st)) != hipSuccess)
        return e;
      for (const auto& s : scatters)
        if ((e = launch_scatter_add(d_colsum + s.col, s.gmap ? d_gmap : nullptr, s.count, d_call, s.which, st)) !=
            hipSuccess)
          return e;
    }
    if (adjoint && has_jac && n_jcols > 0) {
      if ((e = launch_node_jacobian(d_igrad, grad_stride, d_first, n_nodes, d_inv_n, d_colmap, n_jcols, d_call,
                                    jac_ld, st)) != hipSuccess)
        return e;
    }
    return hipSuccess;
  }

  ~Plan() {
    if (done) {
      (void)hipEventSynchronize(done);
      (void)hipEventDestroy(done);
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (owned && arena) (void)hipFree(arena);
  }
};

// Cached graph plans, least recently used first out.  A plan's arena stays
// allocated while it is cached (at C5 about 80 MB), so the cache is bounded;
// an evicted plan is destroyed after its last launch has finished.
constexpr size_t kMaxPlans = 16;
constexpr int kMaxBatchProblems = 64;
std::unordered_map<std::string, std::unique_ptr<Plan>> g_plans;
uint64_t g_plan_clock = 0;

void evict_plans_locked(size_t keep) {
  while (g_plans.size() > keep) {
    auto victim = g_plans.begin();
    for (auto it = g_plans.begin(); it != g_plans.end(); ++it)
      if (it->second->last_use < victim->second->last_use) victim = it;
    g_plans.erase(victim);
  }
}

// Host-side staging buffer: copies are stream-ordered; the host vector is
// pageable, which makes hipMemcpyAsync take its own copy before returning.
struct Upload {
  size_t off;
  std::vector<char> bytes;
};

template <typename T>
void put(std::vector<Upload>& ups, size_t off, const std::vector<T>& v) {
  Upload u;
  u.off = off;
  u.bytes.resize(v.size() * sizeof(T));
  if (!v.empty()) std::memcpy(u.bytes.data(), v.data(), u.bytes.size());
  ups.push_back(std::move(u));
}

// The call block: CallPtrs, then the staging jobs from the next 16-byte
// boundary.  Written by a host-to-device copy before every launch.
constexpr size_t kJobsOff = (sizeof(CallPtrs) + 15) & ~(size_t)15;

size_t add_call_block(Arena& A, size_t n_jobs) {
  return A.add(kJobsOff + sizeof(StageJob) * std::max<size_t>(1, n_jobs));
}

std::vector<char> call_block_image(const CallPtrs& cp, const std::vector<StageJob>& jobs) {
  std::vector<char> b(kJobsOff + sizeof(StageJob) * jobs.size(), 0);
  std::memcpy(b.data(), &cp, sizeof(cp));
  if (!jobs.empty()) std::memcpy(b.data() + kJobsOff, jobs.data(), sizeof(StageJob) * jobs.size());
  return b;
}

template <typename T>
void key_add(std::string& k, const T& v) {
  k.append(reinterpret_cast<const char*>(&v), sizeof(T));
}

// The structure of a coefficient function (not where its coefficients live:
// those are read through the staging jobs of the call block).
void key_fun(std::string& k, const pdd_fun& F) {
  key_add(k, F.n_terms);
  key_add(k, F.n_factors);
  if (F.n_terms > 0 && F.n_factors > 0)
    k.append(reinterpret_cast<const char*>(F.factors), sizeof(pdd_factor) * (size_t)F.n_terms * F.n_factors);
  key_add(k, F.poly_degree);
}

// Estimated mean exit time (in steps) from a node; used only to order work
// items longest first.
double est_steps(const pdd_linear_problem& P, const double* x, double dt) {
  const pdd_domain& D = P.domain;
  const double s2 = P.sigma * P.sigma;
  double tau;
  if (D.kind == PDD_DOM_BALL) {
    double r2 = 0;
    for (int k = 0; k < D.dim; ++k) r2 += (x[k] - D.center[k]) * (x[k] - D.center[k]);
    tau = std::max(0.0, D.radius * D.radius - r2) / (D.dim * s2);
  } else {
    tau = 1e300;
    for (int k = 0; k < D.dim; ++k) tau = std::min(tau, std::max(0.0, (x[k] - D.lo[k]) * (D.hi[k] - x[k])) / s2);
  }
  return 1.0 + tau / dt;
}

struct Items {
  std::vector<WorkItem> q;        // queue order
  std::vector<int64_t> first;     // per node: first slot
  std::vector<int32_t> slot_node; // per slot: node
};

// Work items, guided sizes.  A node's paths are cut into items of `chunk`
// paths, except about its last eighth, which is cut into items of chunk / 8
// (at least 256) queued after every large item.  While an item's last paths
// finish, the lanes that ran its earlier paths idle; large items make that
// rare, and the small items at the end of the queue even out the finishing
// times of the wavefronts.  Slots stay node-major (a node's items are
// consecutive), so per-node reductions run in a fixed order.  Within each
// size class the queue is ordered longest first by `cost` when given.
Items make_items(int64_t n_nodes, const int64_t* counts, int64_t count_all, int chunk, const std::vector<double>& cost) {
  Items r;
  r.first.resize((size_t)n_nodes + 1);
  const int64_t big = std::max(1, chunk);
  const int64_t small = std::max<int64_t>(std::min<int64_t>(256, big), big / 8);
  std::vector<WorkItem> slots;
  std::vector<char> is_small;
  for (int64_t i = 0; i < n_nodes; ++i) {
    r.first[(size_t)i] = (int64_t)slots.size();
    const int64_t N = counts ? counts[i] : count_all;
    const int64_t n_big = N > big ? (N - N / 8) / big : 0;
    int64_t p0 = 0;
    auto push = [&](int64_t cnt, bool sm) {
      WorkItem w;
      w.node = (int32_t)i;
      w.p0 = (uint32_t)p0;
      w.count = (uint32_t)cnt;
      w.slot = (int32_t)slots.size();
      slots.push_back(w);
      is_small.push_back(sm ? 1 : 0);
      r.slot_node.push_back((int32_t)i);
      p0 += cnt;
    };
    for (int64_t b = 0; b < n_big; ++b) push(big, false);
    while (p0 < N) push(std::min<int64_t>(small, N - p0), true);
  }
  r.first[(size_t)n_nodes] = (int64_t)slots.size();
  r.q = slots;
  std::stable_sort(r.q.begin(), r.q.end(), [&](const WorkItem& a, const WorkItem& b) {
    const char sa = is_small[(size_t)a.slot], sb = is_small[(size_t)b.slot];
    if (sa != sb) return sa < sb;
    if (cost.empty()) return false;
    return cost[(size_t)a.node] * a.count > cost[(size_t)b.node] * b.count;
  });
  return r;
}

}  // namespace

// ============================================================================= linear walk
namespace {

struct LinearPlanArgs {
  const pdd_linear_problem* P;
  const double* nodes;
  int64_t n_nodes;
  const int64_t* paths;
  double dt;
  uint64_t seed;
  pdd_options opt;
  pdd_node_stat* out;
  bool adjoint;
  const double* w;
  const pdd_fun_grad* grads;
  double* jac;          // value+Jacobian mode: [n_nodes][jac_ld]
  int64_t jac_ld;
  bool wos = false;     // walk on spheres; dt holds eps
  void* fixed = nullptr;     // caller-provided scratch area: no allocation, no graph, no
  size_t fixed_bytes = 0;    // runtime-compiled kernel
};

int64_t param_count(const pdd_linear_problem& P) {
  const int d = P.domain.dim;
  return (int64_t)P.g.n_terms + n_mono(d, P.g.poly_degree) + P.f.n_terms + n_mono(d, P.f.poly_degree) +
         P.c.n_terms + n_mono(d, P.c.poly_degree);
}

pdd_status validate_linear(const LinearPlanArgs& a) {
  if (a.P == nullptr) return fail(PDD_ERR_INVALID_ARG, "problem is NULL");
  const pdd_linear_problem& P = *a.P;
  const pdd_domain& D = P.domain;
  if (D.dim < 1 || D.dim > 3) return fail(PDD_ERR_INVALID_ARG, "domain.dim must be 1..3");
  if (D.kind == PDD_DOM_FREE) return fail(PDD_ERR_INVALID_ARG, "the linear walk needs a bounded domain (BOX or BALL)");
  if (D.kind != PDD_DOM_BOX && D.kind != PDD_DOM_BALL) return fail(PDD_ERR_INVALID_ARG, "unknown domain kind");
  if (D.kind == PDD_DOM_BOX)
    for (int k = 0; k < D.dim; ++k)
      if (!(D.lo[k] < D.hi[k]) || !std::isfinite(D.lo[k]) || !std::isfinite(D.hi[k]))
        return fail(PDD_ERR_INVALID_ARG, "box needs finite lo < hi");
  if (D.kind == PDD_DOM_BALL && !(D.radius > 0.0 && std::isfinite(D.radius)))
    return fail(PDD_ERR_INVALID_ARG, "ball radius must be positive");
  if (!(P.sigma > 0.0) || !std::isfinite(P.sigma)) return fail(PDD_ERR_INVALID_ARG, "sigma must be positive");
  if (!(a.dt > 0.0) || !std::isfinite(a.dt)) return fail(PDD_ERR_INVALID_ARG, "dt must be positive");
  if (a.n_nodes < 0 || a.n_nodes > (int64_t)1 << 30) return fail(PDD_ERR_INVALID_ARG, "n_nodes out of range");
  if (a.n_nodes > 0 && a.paths == nullptr) return fail(PDD_ERR_INVALID_ARG, "paths_host is NULL");
  for (int64_t i = 0; i < a.n_nodes; ++i)
    if (a.paths[i] < 0 || a.paths[i] > (int64_t)0x7FFFFFFF)
      return fail(PDD_ERR_INVALID_ARG, "paths per node must be in [0, 2^31)");
  pdd_status s;
  const int mt_bcf = a.adjoint ? kAdjTerms : 16;
  for (int k = 0; k < D.dim; ++k)
    if ((s = check_fun(P.b[k], D.dim, "b", 16, kMaxPolyBCF)) != PDD_OK) return s;
  if ((s = check_fun(P.c, D.dim, "c", mt_bcf, kMaxPolyBCF)) != PDD_OK) return s;
  if ((s = check_fun(P.f, D.dim, "f", mt_bcf, kMaxPolyBCF)) != PDD_OK) return s;
  if ((s = check_fun(P.g, D.dim, "g", a.adjoint ? kAdjTerms : kMaxTerms, kMaxPolyG)) != PDD_OK) return s;
  const pdd_options& o = a.opt;
  if (o.precision < PDD_FP64_PLAIN || o.precision > PDD_FP32_STEP) return fail(PDD_ERR_INVALID_ARG, "unknown precision");
  if (o.rng_layout != PDD_RNG_PAIR52 && o.rng_layout != PDD_RNG_QUAD24) return fail(PDD_ERR_INVALID_ARG, "unknown rng layout");
  if (o.precision == PDD_FP32_STEP && o.rng_layout != PDD_RNG_QUAD24)
    return fail(PDD_ERR_INVALID_ARG, "FP32 stepping requires the QUAD24 layout");
  if (o.max_steps < 0 || o.max_steps > 0x7FFFFFFF) return fail(PDD_ERR_INVALID_ARG, "max_steps out of range");
  if (o.chunk_paths < 0 || o.blocks_per_cu < 0 || o.blocks_per_cu > 64 || o.refill_groups < 0 || o.refill_groups > 64)
    return fail(PDD_ERR_INVALID_ARG, "schedule override out of range");
  if (o.schedule < PDD_SCHED_AUTO || o.schedule > PDD_SCHED_PERSISTENT_GRAPH) return fail(PDD_ERR_INVALID_ARG, "unknown schedule");
  if (o.boundary_correction < 0 || o.boundary_correction > 1)
    return fail(PDD_ERR_INVALID_ARG, "boundary_correction must be 0 or 1");
  if (o.specialize < -1 || o.specialize > 1) return fail(PDD_ERR_INVALID_ARG, "specialize must be -1, 0 or 1");
  if (o.skip_items || o.partials) {
    if (a.adjoint || o.precision == PDD_FP64_PLAIN)
      return fail(PDD_ERR_UNSUPPORTED, "skip_items / partials apply to the batched forward walk only");
    if (o.skip_items && !o.partials) return fail(PDD_ERR_INVALID_ARG, "skip_items needs partials");
    if (o.partials && a.n_nodes > 0) {
      pdd_status s2 = check_device_ptr(o.partials, "options->partials");
      if (s2 != PDD_OK) return s2;
    }
  }
  if (a.wos) {
    auto zero = [](const pdd_fun& F) { return F.n_terms == 0 && F.poly_degree < 0; };
    bool ok = zero(P.c) && zero(P.f);
    for (int k = 0; k < D.dim; ++k) ok = ok && zero(P.b[k]);
    if (!ok) return fail(PDD_ERR_UNSUPPORTED, "walk on spheres needs b = c = f = 0 (Laplace's equation)");
    if (o.precision == PDD_FP64_PLAIN) return fail(PDD_ERR_UNSUPPORTED, "walk on spheres has no plain variant");
    if (o.boundary_correction) return fail(PDD_ERR_INVALID_ARG, "boundary_correction does not apply to walk on spheres");
  }
  if (a.n_nodes > 0) {
    if ((s = check_device_ptr(a.nodes, "nodes_dev")) != PDD_OK) return s;
    if (!a.adjoint || a.out || a.jac) if ((s = check_device_ptr(a.out, "out_dev")) != PDD_OK) return s;
    if (a.adjoint && !a.jac && (s = check_device_ptr(a.w, "w_dev")) != PDD_OK) return s;
    if (a.jac && (s = check_device_ptr(a.jac, "jac_dev")) != PDD_OK) return s;
  }
  if (a.jac && a.jac_ld < param_count(P)) return fail(PDD_ERR_INVALID_ARG, "jac_ld is smaller than pdd_param_count");
  if ((o.dump_phi || o.dump_steps) && a.adjoint && o.precision == PDD_FP64_PLAIN)
    return fail(PDD_ERR_UNSUPPORTED, "per-path dumps are not produced by the plain adjoint");
  if (o.dump_steps && !o.dump_phi) return fail(PDD_ERR_INVALID_ARG, "dump_steps needs dump_phi");
  if (a.adjoint) {
    if (a.grads == nullptr && a.jac == nullptr) return fail(PDD_ERR_INVALID_ARG, "grads_host is NULL");
  }
  return PDD_OK;
}

// The device record of one linear problem (domain, exit-test domain, step,
// sigma sqrt(dt), censoring cap, seed, where its functions' data sit in the
// staged tables T); b, c, f polynomials are padded to degree dfc.
void fill_linear_params(const pdd_linear_problem& P, double dt, const pdd_options& o, bool wos, uint64_t seed,
                        int dfc, Tables& T, LinearParams& lp) {
  const int dim = P.domain.dim;
  lp.dim = dim;
  lp.dom_kind = P.domain.kind;
  lp.layout = o.rng_layout;
  for (int k = 0; k < 3; ++k) {
    lp.lo[k] = P.domain.lo[k]; lp.hi[k] = P.domain.hi[k]; lp.ctr[k] = P.domain.center[k];
    lp.lof[k] = (float)lp.lo[k]; lp.hif[k] = (float)lp.hi[k]; lp.ctrf[k] = (float)lp.ctr[k];
  }
  lp.rad = P.domain.radius;
  lp.rad2 = P.domain.radius * P.domain.radius;
  lp.radf = (float)lp.rad;
  lp.rad2f = (float)lp.rad2;
  // exit-test domain: D, or D shrunk by c0 sigma sqrt(dt) (Gobet-Menozzi shift;
  // c0 = -zeta(1/2)/sqrt(2 pi), zeta(1/2) = -1.4603545088095868...)
  {
    const double delta = o.boundary_correction ? (1.4603545088095868 / std::sqrt(2.0 * M_PI)) * P.sigma * std::sqrt(dt)
                                               : 0.0;
    double trad = P.domain.radius - delta;
    if (trad < 0.0) trad = 0.0;
    for (int k = 0; k < 3; ++k) {
      lp.tlo[k] = P.domain.lo[k] + delta;
      lp.thi[k] = P.domain.hi[k] - delta;
      lp.tlof[k] = (float)lp.tlo[k];
      lp.thif[k] = (float)lp.thi[k];
    }
    lp.trad2 = trad * trad;
    lp.trad2f = (float)lp.trad2;
  }
  lp.dt = dt;
  lp.sdt = P.sigma * std::sqrt(dt);
  lp.dtf = (float)lp.dt;
  lp.sdtf = (float)lp.sdt;
  lp.max_steps = o.max_steps > 0 ? o.max_steps : (wos ? (int64_t)100000 : (int64_t)std::ceil(100.0 / dt));
  if (lp.max_steps > 0x7FFFFFFF) lp.max_steps = 0x7FFFFFFF;
  lp.key0 = (uint32_t)seed;
  lp.key1 = (uint32_t)(seed >> 32);
  pdd_fun zero{};
  zero.poly_degree = -1;
  for (int k = 0; k < 3; ++k) lp.b[k] = T.add(k < dim ? P.b[k] : zero, dim, dfc, false, k);
  lp.c = T.add(P.c, dim, dfc, false, 3);
  lp.f = T.add(P.f, dim, dfc, false, 4);
  lp.g = T.add(P.g, dim, 0, true, 5);
  lp.n_fac = (int)T.fac.size();
  auto nonzero = [](const DevFun& F) { return F.n_terms > 0 || F.poly_deg >= 0; };
  lp.has_b = nonzero(lp.b[0]) || nonzero(lp.b[1]) || nonzero(lp.b[2]);
  lp.has_c = nonzero(lp.c);
  lp.has_f = nonzero(lp.f);
}

// Captures a plan's launches into a graph (the uploads were ordered before
// on the caller's stream; the capture runs on a private stream that first
// waits for them), launches it once and caches it under `key`.
pdd_status capture_plan(std::unique_ptr<Plan> plan, const std::string& key, hipStream_t st) {
  Plan& pl = *plan;
  hipStream_t cap;
  PDD_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  hipEvent_t ready;
  PDD_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
  PDD_HIP(hipEventRecord(ready, st));
  PDD_HIP(hipStreamWaitEvent(cap, ready, 0));
  PDD_HIP(hipStreamSynchronize(cap));
  PDD_HIP(hipEventDestroy(ready));
  PDD_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
  hipError_t e = pl.enqueue(cap);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(cap, &g);
  (void)hipStreamDestroy(cap);
  if (e != hipSuccess || e2 != hipSuccess)
    return fail(PDD_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
  pl.graph = g;
  PDD_HIP(hipGraphInstantiate(&pl.exec, g, nullptr, nullptr, 0));
  PDD_HIP(hipEventCreateWithFlags(&pl.done, hipEventDisableTiming));
  PDD_HIP(hipGraphLaunch(pl.exec, st));
  PDD_HIP(hipEventRecord(pl.done, st));
  std::lock_guard<std::mutex> lk(g_mu);
  pl.last_use = ++g_plan_clock;
  evict_plans_locked(kMaxPlans - 1);
  g_plans[key] = std::move(plan);
  return PDD_OK;
}

const double* job_source(const pdd_linear_problem& P, const double* nodes, JobSource js) {
  if (js.part == 3) return nodes;
  if (js.part == 2 || js.fun < 0) return nullptr;
  const pdd_fun& F = js.fun < 3 ? P.b[js.fun] : (js.fun == 3 ? P.c : (js.fun == 4 ? P.f : P.g));
  return js.part == 0 ? F.coef : F.poly;
}

CallPtrs call_ptrs(const LinearPlanArgs& a) {
  CallPtrs c{};
  c.out = a.out;
  c.w = a.w;
  c.jac = a.jac;
  if (a.adjoint && a.grads != nullptr)
    for (int k = 0; k < 3; ++k) {
      c.grad[2 * k] = a.grads[k].dcoef;
      c.grad[2 * k + 1] = a.grads[k].dpoly;
    }
  return c;
}

pdd_status run_linear(const LinearPlanArgs& a, hipStream_t st) {
  pdd_status s = validate_linear(a);
  if (s != PDD_OK) return s;
  if (a.n_nodes == 0) return PDD_OK;  // nothing to enqueue (gradients stay as they are)
  const pdd_linear_problem& P = *a.P;
  const int dim = P.domain.dim;
  const pdd_options& o = a.opt;
  const bool plain = o.precision == PDD_FP64_PLAIN;
  const bool fp32 = o.precision == PDD_FP32_STEP;
  const bool graph = !plain && (o.schedule == PDD_SCHED_AUTO || o.schedule == PDD_SCHED_PERSISTENT_GRAPH) &&
                     o.dump_phi == nullptr && o.skip_items == nullptr && o.partials == nullptr &&
                     a.fixed == nullptr;

  // ---- plan cache lookup: the key holds what shapes the launch (problem
  // structure, budgets, step, seed, options, which outputs are wanted, the
  // stream), not the caller's buffers, which reach a replay through the call
  // block
  std::string key;
  if (graph) {
    key_add(key, a.adjoint ? 2 : (a.wos ? 3 : 1));
    int dev = 0;
    PDD_HIP(hipGetDevice(&dev));
    key_add(key, dev);
    key_add(key, st);
    key_add(key, P.domain);
    key_add(key, P.sigma);
    for (int k = 0; k < 3; ++k) key_fun(key, P.b[k]);
    key_fun(key, P.c);
    key_fun(key, P.f);
    key_fun(key, P.g);
    key_add(key, a.n_nodes);
    key.append(reinterpret_cast<const char*>(a.paths), sizeof(int64_t) * (size_t)a.n_nodes);
    key_add(key, a.dt);
    key_add(key, a.seed);
    key_add(key, o);
    const CallPtrs cp = call_ptrs(a);
    uint32_t present = (cp.out ? 1u : 0u) | (cp.w ? 2u : 0u) | (cp.jac ? 4u : 0u);
    for (int k = 0; k < 6; ++k) present |= cp.grad[k] ? (8u << k) : 0u;
    key_add(key, present);
    key_add(key, a.jac_ld);
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_plans.find(key);
    if (it != g_plans.end()) {
      Plan& hp = *it->second;
      hp.last_use = ++g_plan_clock;
      std::vector<StageJob> jobs = hp.jobs_host;
      for (size_t j = 0; j < jobs.size(); ++j) jobs[j].src = job_source(P, a.nodes, hp.job_src[j]);
      const std::vector<char> img = call_block_image(cp, jobs);
      PDD_HIP(hipMemcpyAsync(hp.d_call, img.data(), img.size(), hipMemcpyHostToDevice, st));
      PDD_HIP(hipGraphLaunch(hp.exec, st));
      PDD_HIP(hipEventRecord(hp.done, st));
      return PDD_OK;
    }
  }

  std::unique_ptr<Plan> plan(new Plan());
  Plan& pl = *plan;
  pl.plain = plain;
  pl.adjoint = a.adjoint;
  PDD_HIP(hipGetDevice(&pl.device));
  if ((s = counters(&pl.ctr)) != PDD_OK) return s;

  // ---- tables
  const bool any_poly = P.c.poly_degree >= 0 || P.f.poly_degree >= 0 || P.b[0].poly_degree >= 0 ||
                        (dim > 1 && P.b[1].poly_degree >= 0) || (dim > 2 && P.b[2].poly_degree >= 0);
  const int dfc = any_poly ? kMaxPolyBCF : -1;
  Tables T;
  LinearParams& lp = pl.lp;
  fill_linear_params(P, a.dt, o, a.wos, a.seed, dfc, T, lp);

  // ---- work items
  int64_t total_paths = 0;
  for (int64_t i = 0; i < a.n_nodes; ++i) total_paths += a.paths[i];
  const int kernel = a.adjoint ? PDD_KERNEL_WALK_ADJOINT : (a.wos ? PDD_KERNEL_WOS : PDD_KERNEL_WALK);
  const Tuning tune = choose_schedule(kernel, dim, fp32 ? PDD_FP32_STEP : PDD_FP64, o, device_cus(), total_paths);
  std::vector<double> cost((size_t)a.n_nodes);
  for (int64_t i = 0; i < a.n_nodes; ++i) cost[(size_t)i] = 0.0;
  std::vector<double> hnodes((size_t)a.n_nodes * dim);
  if (a.n_nodes > 0) {
    PDD_HIP(hipMemcpyAsync(hnodes.data(), a.nodes, hnodes.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    PDD_HIP(hipStreamSynchronize(st));
    for (int64_t i = 0; i < a.n_nodes; ++i) cost[(size_t)i] = est_steps(P, &hnodes[(size_t)i * dim], a.dt);
  }
  Items items;
  std::vector<int64_t> plain_first;
  std::vector<PlainLaunch> plain_launches;
  int n_slots = 0;
  if (!plain) {
    items = make_items(a.n_nodes, a.paths, 0, tune.chunk_paths, cost);
    n_slots = (int)items.q.size();
    if (o.skip_items) {
      // resume: queue only the items not skipped; all slots stay in place
      std::vector<WorkItem> keep;
      for (const WorkItem& w : items.q)
        if (!o.skip_items[w.slot]) keep.push_back(w);
      items.q.swap(keep);
    }
  }
  int n_items = (int)items.q.size();
  pl.n_items = n_items;
  pl.n_nodes = a.n_nodes;

  // ---- arena layout
  Arena A;
  const size_t o_call = add_call_block(A, T.jobs.size() + 1);   // + the node-coordinate job
  const size_t o_nodes = A.add(sizeof(double) * (size_t)a.n_nodes * (size_t)dim);
  const size_t o_perm = A.add(sizeof(int32_t) * std::max<size_t>(1, T.perm.size()));
  const size_t o_fac = A.add(sizeof(DevFactor) * std::max<size_t>(1, T.fac.size()));
  const size_t o_cd = A.add(sizeof(double) * std::max(1, T.ncoef));
  const size_t o_cf = A.add(sizeof(float) * std::max(1, T.ncoef));
  const size_t o_q = A.add(sizeof(uint32_t) * 4);
  size_t o_items = 0, o_istat = 0, o_first = 0, o_doff = 0;
  std::vector<int64_t> doff((size_t)a.n_nodes + 1, 0);
  for (int64_t i = 0; i < a.n_nodes; ++i) doff[(size_t)i + 1] = doff[(size_t)i] + a.paths[i];
  int64_t n_stat = 0;
  if (plain) {
    // forward: at most 4096 grid-striding blocks per node; adjoint: one path
    // per thread, one derivative row per block
    plain_first.resize((size_t)a.n_nodes + 1);
    for (int64_t i = 0; i < a.n_nodes; ++i) {
      plain_first[(size_t)i] = n_stat;
      const int64_t N = a.paths[i];
      const int64_t nb = std::max<int64_t>(1, a.adjoint ? (N + kBlock - 1) / kBlock
                                                        : std::min<int64_t>((N + kBlock - 1) / kBlock, 4096));
      n_stat += nb;
      if (a.adjoint) items.slot_node.insert(items.slot_node.end(), (size_t)nb, (int32_t)i);
    }
    plain_first[(size_t)a.n_nodes] = n_stat;
    if (a.adjoint) {
      items.first = plain_first;
      n_items = (int)n_stat;
      pl.n_items = n_items;
    }
  } else {
    n_stat = n_slots;
    o_items = A.add(sizeof(WorkItem) * std::max(1, n_items));
  }
  o_istat = A.add(sizeof(ItemStat) * std::max<int64_t>(1, n_stat));
  o_first = A.add(sizeof(int64_t) * ((size_t)a.n_nodes + 1));
  o_doff = A.add(sizeof(int64_t) * ((size_t)a.n_nodes + 1));
  // adjoint buffers
  const int NM = dfc >= 0 ? n_mono(dim, dfc) : 0;
  // generic terms anywhere in b, c, f select the term-capable kernels; for the
  // adjoint (terms in b, c, f or g) the rows then carry kAdjTerms term
  // columns per function
  bool bcf_terms = P.c.n_terms > 0 || P.f.n_terms > 0;
  for (int k = 0; k < dim; ++k) bcf_terms = bcf_terms || P.b[k].n_terms > 0;
  const bool terms = a.adjoint ? (bcf_terms || P.g.n_terms > 0) : bcf_terms;
  const int nt = (a.adjoint && terms) ? kAdjTerms : 0;
  const int NP = nt + NM;
  const int ngm = lp.g.poly_deg >= 0 ? lp.g.n_mono : 0;
  size_t o_igrad = 0, o_slot = 0, o_invn = 0, o_col = 0, o_gmap = 0;
  std::vector<int32_t> gmap;
  if (a.adjoint) {
    pl.grad_stride = nt + ngm + 2 * NP;
    o_igrad = A.add(sizeof(double) * (size_t)std::max(1, n_items) * (size_t)pl.grad_stride);
    o_slot = A.add(sizeof(int32_t) * std::max(1, n_items));
    o_invn = A.add(sizeof(double) * std::max<int64_t>(1, a.n_nodes));
    o_col = A.add(sizeof(double) * std::max(1, pl.grad_stride));
    if (ngm > 0) gmap = nested_to_graded(dim, lp.g.poly_deg);
    o_gmap = A.add(sizeof(int32_t) * std::max<size_t>(1, gmap.size()));
  }
  // Jacobian columns (caller order) -> per-item row columns
  std::vector<int32_t> colmap;
  size_t o_colmap = 0;
  if (a.jac) {
    std::vector<int32_t> graded_to_nested(gmap.size());
    for (size_t j = 0; j < gmap.size(); ++j) graded_to_nested[(size_t)gmap[j]] = (int32_t)j;
    for (int t = 0; t < P.g.n_terms; ++t) colmap.push_back(t);
    for (int m = 0; m < ngm; ++m) colmap.push_back(nt + graded_to_nested[(size_t)m]);
    for (int t = 0; t < P.f.n_terms; ++t) colmap.push_back(nt + ngm + t);
    for (int m = 0; m < n_mono(dim, P.f.poly_degree); ++m) colmap.push_back(nt + ngm + nt + m);
    for (int t = 0; t < P.c.n_terms; ++t) colmap.push_back(nt + ngm + NP + t);
    for (int m = 0; m < n_mono(dim, P.c.poly_degree); ++m) colmap.push_back(nt + ngm + NP + nt + m);
    o_colmap = A.add(sizeof(int32_t) * std::max<size_t>(1, colmap.size()));
  }

  // ---- problem-specialised kernel for per-step generic terms
  hipFunction_t spec = nullptr;
  if (!plain && bcf_terms && !a.wos && o.specialize >= 0 && a.fixed == nullptr) {
    const std::string src = spec_terms_source(lp, T.fac);
    std::string why = "a scale or shift is not finite";
    if (src.empty() ||
        !spec_walk_kernel(src, fp32, dim, dfc, fp32 ? (int)PDD_RNG_QUAD24 : o.rng_layout, a.adjoint, &spec, &why)) {
      spec = nullptr;
      if (o.specialize == 1) return fail(PDD_ERR_HIP, "problem-specialised kernel: " + why);
      static std::once_flag once;
      std::call_once(once, [&] {
        std::fprintf(stderr, "pdd: problem-specialised kernel unavailable, using the table-driven kernel: %s\n",
                     why.c_str());
      });
    }
  }

  // ---- allocate
  ArenaLease lease;
  if (a.fixed != nullptr) {
    if (A.total > a.fixed_bytes)
      return fail(PDD_ERR_UNSUPPORTED, "this call needs " + std::to_string(A.total) +
                                           " bytes of scratch; the fixed scratch area holds " +
                                           std::to_string(a.fixed_bytes));
    pl.arena = a.fixed;
  } else if (graph) {
    PDD_HIP(hipMalloc(&pl.arena, A.total));
    pl.owned = true;
  } else {
    PDD_HIP(lease_arena(A.total, st, &lease, &pl.arena));
  }
  char* base = (char*)pl.arena;
  pl.d_call = (CallPtrs*)(base + o_call);
  pl.d_jobs = (StageJob*)(base + o_call + kJobsOff);
  pl.d_nodes = (double*)(base + o_nodes);
  T.job(StageJob{a.nodes, pl.d_nodes, 0, (int32_t)(a.n_nodes * dim), -1, 0}, -1, 3);
  pl.n_jobs = (int)T.jobs.size();
  pl.jobs_host = T.jobs;
  pl.job_src = T.src;
  pl.d_perm = (int32_t*)(base + o_perm);
  DevFactor* d_fac = (DevFactor*)(base + o_fac);
  pl.d_cd = (double*)(base + o_cd);
  pl.d_cf = (float*)(base + o_cf);
  pl.d_qhead = (uint32_t*)(base + o_q);
  pl.d_istat = o.partials ? (ItemStat*)o.partials : (ItemStat*)(base + o_istat);
  pl.d_first = (int64_t*)(base + o_first);
  int64_t* d_doff = (int64_t*)(base + o_doff);
  pl.has_out = a.out != nullptr;
  lp.fac = d_fac;
  lp.cd = pl.d_cd;
  lp.cf = pl.d_cf;
  lp.nodes = pl.d_nodes;

  std::vector<Upload> ups;
  put(ups, o_call, call_block_image(call_ptrs(a), T.jobs));
  put(ups, o_perm, T.perm);
  put(ups, o_fac, T.fac);
  put(ups, o_doff, doff);
  if (plain) {
    put(ups, o_first, plain_first);
  } else {
    put(ups, o_first, items.first);
    put(ups, o_items, items.q);
  }
  if (a.adjoint) {
    std::vector<double> invn((size_t)std::max<int64_t>(1, a.n_nodes), 0.0);
    for (int64_t i = 0; i < a.n_nodes; ++i) invn[(size_t)i] = a.paths[i] > 0 ? 1.0 / (double)a.paths[i] : 0.0;
    put(ups, o_slot, items.slot_node);
    put(ups, o_invn, invn);
    if (!gmap.empty()) put(ups, o_gmap, gmap);
    pl.d_igrad = (double*)(base + o_igrad);
    pl.d_slot_node = (int32_t*)(base + o_slot);
    pl.d_inv_n = (double*)(base + o_invn);
    pl.d_colsum = (double*)(base + o_col);
    pl.d_gmap = (int32_t*)(base + o_gmap);
    pl.has_w = a.w != nullptr;
    if (a.jac) {
      put(ups, o_colmap, colmap);
      pl.d_colmap = (int32_t*)(base + o_colmap);
      pl.has_jac = true;
      pl.jac_ld = a.jac_ld;
      pl.n_jcols = (int)colmap.size();
    }
  }
  if (a.adjoint && a.grads != nullptr && a.w != nullptr) {
    // scatter of reduced columns into the caller's arrays
    const pdd_fun_grad& gg = a.grads[0];
    const pdd_fun_grad& gf = a.grads[1];
    const pdd_fun_grad& gc = a.grads[2];
    int col = 0;
    if (gg.dcoef && P.g.n_terms > 0) pl.scatters.push_back({col, P.g.n_terms, false, 0});
    col += nt;
    if (gg.dpoly && ngm > 0) pl.scatters.push_back({col, ngm, true, 1});
    col += ngm;
    if (gf.dcoef && P.f.n_terms > 0) pl.scatters.push_back({col, P.f.n_terms, false, 2});
    if (gf.dpoly && P.f.poly_degree >= 0) pl.scatters.push_back({col + nt, n_mono(dim, P.f.poly_degree), false, 3});
    col += NP;
    if (gc.dcoef && P.c.n_terms > 0) pl.scatters.push_back({col, P.c.n_terms, false, 4});
    if (gc.dpoly && P.c.poly_degree >= 0) pl.scatters.push_back({col + nt, n_mono(dim, P.c.poly_degree), false, 5});
  }
  for (const auto& u : ups)
    if (!u.bytes.empty()) PDD_HIP(hipMemcpyAsync(base + u.off, u.bytes.data(), u.bytes.size(), hipMemcpyHostToDevice, st));

  // ---- launch descriptors
  if (plain) {
    for (int64_t i = 0; i < a.n_nodes; ++i) {
      PlainLaunch L{};
      L.P = &pl.lp;
      L.dfc = dfc;
      L.grid = (int)(plain_first[(size_t)i + 1] - plain_first[(size_t)i]);
      L.node = (int)i;
      L.n_paths = (uint32_t)a.paths[i];
      L.bstat = pl.d_istat + plain_first[(size_t)i];
      L.dump_phi = o.dump_phi;
      L.dump_steps = o.dump_steps;
      L.dump_base = doff[(size_t)i];
      L.adjoint = a.adjoint;
      L.nt = nt;
      L.brow = a.adjoint ? pl.d_igrad + (size_t)plain_first[(size_t)i] * (size_t)pl.grad_stride : nullptr;
      L.grad_stride = pl.grad_stride;
      pl.pl.push_back(L);
    }
  } else {
    WalkLaunch& L = pl.wl;
    L.P = &pl.lp;
    L.dfc = dfc;
    L.terms = terms;
    L.fp32 = fp32;
    L.adjoint = a.adjoint;
    L.wos = a.wos;
    L.spec = spec;
    const int max_blocks = tune.blocks_per_cu * device_cus();
    const int need = (n_items + kBlock / kWave - 1) / (kBlock / kWave);
    L.grid = std::max(1, std::min(max_blocks, need));
    L.items = (const WorkItem*)(base + o_items);
    L.n_items = n_items;
    L.qhead = pl.d_qhead;
    L.istat = pl.d_istat;
    L.igrad = pl.d_igrad;
    L.grad_stride = pl.grad_stride;
    L.dump_phi = o.dump_phi;
    L.dump_steps = o.dump_steps;
    L.dump_off = d_doff;
    L.refill_groups = tune.refill_groups;
  }

  // ---- run
  if (!graph) {
    hipError_t e = pl.enqueue(st);
    (void)lease.done();
    if (e != hipSuccess) return fail(PDD_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
    return PDD_OK;
  }
  return capture_plan(std::move(plan), key, st);
}

// ---------------------------------------------------------------------------- batch of problems
struct BatchArgs {
  const pdd_linear_problem* probs;
  int32_t n_probs;
  const int32_t* node_prob;   // host [n_nodes]
  const double* nodes;        // device [n_nodes][3]
  int64_t n_nodes;
  const int64_t* paths;
  double dt;                  // Euler step, or the walk-on-spheres shell width
  uint64_t seed;
  pdd_options opt;
  pdd_node_stat* out;
  bool wos;
};

pdd_status run_linear_batch(const BatchArgs& a, hipStream_t st) {
  if (a.probs == nullptr) return fail(PDD_ERR_INVALID_ARG, "problems is NULL");
  if (a.n_probs < 1 || a.n_probs > kMaxBatchProblems)
    return fail(PDD_ERR_INVALID_ARG, "n_problems must be 1.." + std::to_string(kMaxBatchProblems));
  const pdd_options& o = a.opt;
  pdd_status s;
  for (int k = 0; k < a.n_probs; ++k) {
    LinearPlanArgs v{&a.probs[k], nullptr, 0, nullptr, a.dt, a.seed, o, a.out, false, nullptr, nullptr, nullptr, 0};
    v.wos = a.wos;
    if ((s = validate_linear(v)) != PDD_OK) return fail(s, "problem " + std::to_string(k) + ": " + pdd_last_error());
    const pdd_linear_problem& P = a.probs[k];
    bool terms = P.c.n_terms > 0 || P.f.n_terms > 0;
    for (int d = 0; d < P.domain.dim; ++d) terms = terms || P.b[d].n_terms > 0;
    if (terms)
      return fail(PDD_ERR_UNSUPPORTED, "problem " + std::to_string(k) +
                                           ": the batch takes b, c, f as dense polynomials (no generic terms)");
  }
  if (o.precision == PDD_FP64_PLAIN) return fail(PDD_ERR_UNSUPPORTED, "the batch has no plain variant");
  if (o.skip_items || o.partials) return fail(PDD_ERR_UNSUPPORTED, "skip_items / partials: single-problem calls only");
  if (a.n_nodes < 0 || a.n_nodes > (int64_t)1 << 30) return fail(PDD_ERR_INVALID_ARG, "n_nodes out of range");
  if (a.n_nodes == 0) return PDD_OK;
  if (a.paths == nullptr || a.node_prob == nullptr) return fail(PDD_ERR_INVALID_ARG, "paths_host or node_problem is NULL");
  int64_t total_paths = 0;
  for (int64_t i = 0; i < a.n_nodes; ++i) {
    if (a.paths[i] < 0 || a.paths[i] > (int64_t)0x7FFFFFFF)
      return fail(PDD_ERR_INVALID_ARG, "paths per node must be in [0, 2^31)");
    if (a.node_prob[i] < 0 || a.node_prob[i] >= a.n_probs)
      return fail(PDD_ERR_INVALID_ARG, "node_problem entry out of range");
    total_paths += a.paths[i];
  }
  if ((s = check_device_ptr(a.nodes, "nodes_dev")) != PDD_OK) return s;
  if ((s = check_device_ptr(a.out, "out_dev")) != PDD_OK) return s;
  const bool fp32 = o.precision == PDD_FP32_STEP;
  const bool graph = (o.schedule == PDD_SCHED_AUTO || o.schedule == PDD_SCHED_PERSISTENT_GRAPH) &&
                     o.dump_phi == nullptr;
  auto sources = [&](const std::vector<StageJob>& tmpl, const std::vector<JobSource>& src) {
    std::vector<StageJob> jobs = tmpl;
    for (size_t j = 0; j < jobs.size(); ++j) jobs[j].src = job_source(a.probs[src[j].prob], a.nodes, src[j]);
    return jobs;
  };
  CallPtrs cp{};
  cp.out = a.out;

  std::string key;
  if (graph) {
    key_add(key, a.wos ? 5 : 4);
    int dev = 0;
    PDD_HIP(hipGetDevice(&dev));
    key_add(key, dev);
    key_add(key, st);
    key_add(key, a.n_probs);
    for (int k = 0; k < a.n_probs; ++k) {
      const pdd_linear_problem& P = a.probs[k];
      key_add(key, P.domain);
      key_add(key, P.sigma);
      for (int d = 0; d < 3; ++d) key_fun(key, P.b[d]);
      key_fun(key, P.c);
      key_fun(key, P.f);
      key_fun(key, P.g);
    }
    key_add(key, a.n_nodes);
    key.append(reinterpret_cast<const char*>(a.node_prob), sizeof(int32_t) * (size_t)a.n_nodes);
    key.append(reinterpret_cast<const char*>(a.paths), sizeof(int64_t) * (size_t)a.n_nodes);
    key_add(key, a.dt);
    key_add(key, a.seed);
    key_add(key, o);
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_plans.find(key);
    if (it != g_plans.end()) {
      Plan& hp = *it->second;
      hp.last_use = ++g_plan_clock;
      const std::vector<char> img = call_block_image(cp, sources(hp.jobs_host, hp.job_src));
      PDD_HIP(hipMemcpyAsync(hp.d_call, img.data(), img.size(), hipMemcpyHostToDevice, st));
      PDD_HIP(hipGraphLaunch(hp.exec, st));
      PDD_HIP(hipEventRecord(hp.done, st));
      return PDD_OK;
    }
  }

  std::unique_ptr<Plan> plan(new Plan());
  Plan& pl = *plan;
  pl.batch = true;
  PDD_HIP(hipGetDevice(&pl.device));
  if ((s = counters(&pl.ctr)) != PDD_OK) return s;

  // ---- per-problem records and the shared tables
  Tables T;
  std::vector<LinearParams> lps((size_t)a.n_probs);
  for (int k = 0; k < a.n_probs; ++k) {
    T.cur_prob = k;
    fill_linear_params(a.probs[k], a.dt, o, a.wos, a.seed, kMaxPolyBCF, T, lps[(size_t)k]);
  }
  T.cur_prob = 0;

  // ---- work items: one queue over every problem's nodes
  const Tuning tune = choose_schedule(a.wos ? PDD_KERNEL_WOS_BATCH : PDD_KERNEL_WALK_BATCH, 0,
                                      fp32 ? PDD_FP32_STEP : PDD_FP64, o, device_cus(), total_paths);
  std::vector<double> hnodes((size_t)a.n_nodes * 3);
  PDD_HIP(hipMemcpyAsync(hnodes.data(), a.nodes, hnodes.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  PDD_HIP(hipStreamSynchronize(st));
  std::vector<double> cost((size_t)a.n_nodes);
  for (int64_t i = 0; i < a.n_nodes; ++i)
    cost[(size_t)i] = est_steps(a.probs[a.node_prob[i]], &hnodes[(size_t)i * 3], a.dt);
  Items items = make_items(a.n_nodes, a.paths, 0, tune.chunk_paths, cost);
  const int n_items = (int)items.q.size();
  pl.n_items = n_items;
  pl.n_nodes = a.n_nodes;
  std::vector<int64_t> doff((size_t)a.n_nodes + 1, 0);
  for (int64_t i = 0; i < a.n_nodes; ++i) doff[(size_t)i + 1] = doff[(size_t)i] + a.paths[i];

  // ---- arena
  Arena A;
  const size_t o_call = add_call_block(A, T.jobs.size() + 1);
  const size_t o_nodes = A.add(sizeof(double) * (size_t)a.n_nodes * 3);
  const size_t o_perm = A.add(sizeof(int32_t) * std::max<size_t>(1, T.perm.size()));
  const size_t o_fac = A.add(sizeof(DevFactor) * std::max<size_t>(1, T.fac.size()));
  const size_t o_cd = A.add(sizeof(double) * std::max(1, T.ncoef));
  const size_t o_cf = A.add(sizeof(float) * std::max(1, T.ncoef));
  const size_t o_q = A.add(sizeof(uint32_t) * 4);
  const size_t o_items = A.add(sizeof(WorkItem) * std::max(1, n_items));
  const size_t o_istat = A.add(sizeof(ItemStat) * std::max(1, n_items));
  const size_t o_first = A.add(sizeof(int64_t) * ((size_t)a.n_nodes + 1));
  const size_t o_doff = A.add(sizeof(int64_t) * ((size_t)a.n_nodes + 1));
  const size_t o_probs = A.add(sizeof(LinearParams) * (size_t)a.n_probs);
  const size_t o_nprob = A.add(sizeof(int32_t) * (size_t)a.n_nodes);
  ArenaLease lease;
  if (graph) {
    PDD_HIP(hipMalloc(&pl.arena, A.total));
    pl.owned = true;
  } else {
    PDD_HIP(lease_arena(A.total, st, &lease, &pl.arena));
  }
  char* base = (char*)pl.arena;
  pl.d_call = (CallPtrs*)(base + o_call);
  pl.d_jobs = (StageJob*)(base + o_call + kJobsOff);
  pl.d_nodes = (double*)(base + o_nodes);
  T.job(StageJob{a.nodes, pl.d_nodes, 0, (int32_t)(a.n_nodes * 3), -1, 0}, -1, 3);
  pl.n_jobs = (int)T.jobs.size();
  pl.jobs_host = T.jobs;
  pl.job_src = T.src;
  pl.d_perm = (int32_t*)(base + o_perm);
  pl.d_cd = (double*)(base + o_cd);
  pl.d_cf = (float*)(base + o_cf);
  pl.d_qhead = (uint32_t*)(base + o_q);
  pl.d_istat = (ItemStat*)(base + o_istat);
  pl.d_first = (int64_t*)(base + o_first);
  pl.has_out = true;
  for (auto& lp : lps) {
    lp.fac = (const DevFactor*)(base + o_fac);
    lp.cd = pl.d_cd;
    lp.cf = pl.d_cf;
    lp.nodes = pl.d_nodes;
  }
  std::vector<int32_t> nprob(a.node_prob, a.node_prob + a.n_nodes);
  std::vector<Upload> ups;
  put(ups, o_call, call_block_image(cp, sources(T.jobs, T.src)));
  put(ups, o_perm, T.perm);
  put(ups, o_fac, T.fac);
  put(ups, o_items, items.q);
  put(ups, o_first, items.first);
  put(ups, o_doff, doff);
  put(ups, o_probs, lps);
  put(ups, o_nprob, nprob);
  for (const auto& u : ups)
    if (!u.bytes.empty()) PDD_HIP(hipMemcpyAsync(base + u.off, u.bytes.data(), u.bytes.size(), hipMemcpyHostToDevice, st));

  WalkBatchLaunch& L = pl.wbl;
  L.probs = (const LinearParams*)(base + o_probs);
  L.node_prob = (const int32_t*)(base + o_nprob);
  L.nodes = pl.d_nodes;
  L.fac = (const DevFactor*)(base + o_fac);
  L.cd = pl.d_cd;
  L.cf = pl.d_cf;
  L.key0 = (uint32_t)a.seed;
  L.key1 = (uint32_t)(a.seed >> 32);
  L.fp32 = fp32;
  L.layout = o.rng_layout;
  L.wos = a.wos;
  const int max_blocks = tune.blocks_per_cu * device_cus();
  const int need = (n_items + kBlock / kWave - 1) / (kBlock / kWave);
  L.grid = std::max(1, std::min(max_blocks, need));
  L.items = (const WorkItem*)(base + o_items);
  L.n_items = n_items;
  L.qhead = pl.d_qhead;
  L.istat = pl.d_istat;
  L.dump_phi = o.dump_phi;
  L.dump_steps = o.dump_steps;
  L.dump_off = (const int64_t*)(base + o_doff);
  L.refill_groups = tune.refill_groups;

  if (!graph) {
    hipError_t e = pl.enqueue(st);
    (void)lease.done();
    if (e != hipSuccess) return fail(PDD_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
    return PDD_OK;
  }
  return capture_plan(std::move(plan), key, st);
}

}  // namespace

namespace pdd {

pdd_status set_error(pdd_status s, const std::string& msg) { return fail(s, msg); }

pdd_status run_linear_fixed(const pdd_linear_problem* problem, const double* nodes_dev, int64_t n_nodes,
                            const int64_t* paths_host, double dt, uint64_t seed, const pdd_options* options,
                            pdd_node_stat* out_dev, void* area, size_t bytes, void* hip_stream) {
  try {
    if (options == nullptr) return fail(PDD_ERR_INVALID_ARG, "options is NULL");
    if (area == nullptr || bytes == 0) return fail(PDD_ERR_INVALID_ARG, "no scratch area");
    LinearPlanArgs a{problem, nodes_dev, n_nodes, paths_host, dt, seed, *options, out_dev, false, nullptr, nullptr,
                     nullptr, 0};
    a.fixed = area;
    a.fixed_bytes = bytes;
    return run_linear(a, (hipStream_t)hip_stream);
  } catch (const std::bad_alloc&) {
    return fail(PDD_ERR_NO_MEMORY, "host allocation failed");
  } catch (...) {
    return fail(PDD_ERR_HIP, "unexpected exception");
  }
}

}  // namespace pdd

// ============================================================================= branching
namespace {

// Assumption 3.2 with l0(s) = sum |alpha_k| s^k, l(s) = beta (l0(s psi_sup)/psi_sup - s):
// admissible if l(1) <= 0, or l has a zero beyond 1, or int_1^inf ds / l(s) > T.
bool admissible_scan(const pdd_branching_problem& B, std::string* why) {
  const double ps = B.psi_sup;
  auto l = [&](double s) {
    double l0 = 0.0, p = 1.0;
    for (int k = 0; k < 5; ++k) {
      l0 += std::fabs(B.alpha[k]) * p;
      p *= s * ps;
    }
    return B.beta * (l0 / ps - s);
  };
  if (l(1.0) <= 0.0) return true;
  // scan for a zero on (1, 1e12] on a log grid; integrate 1/l meanwhile
  const int n = 200000;
  const double lmax = std::log(1e12);
  double integral = 0.0;
  double prev_t = 0.0, prev_f = 1.0 / l(1.0);
  for (int i = 1; i <= n; ++i) {
    const double t = lmax * i / n;
    const double s = std::exp(t);
    const double v = l(s);
    if (v <= 0.0) return true;
    const double f = s / v;  // integrand in t = ln s (ds = s dt)
    integral += 0.5 * (f + prev_f) * (t - prev_t);
    prev_t = t;
    prev_f = f;
  }
  // tail beyond s = 1e12: for l growing at least quadratically it is at most
  // s / l(s) at the last grid point
  integral += prev_f;
  if (integral > B.T) return true;
  if (why) *why = "the branching representation may blow up before T (Assumption 3.2: l(1) > 0 and int 1/l = " +
                  std::to_string(integral) + " <= T)";
  return false;
}

// The scan above depends only on alpha, sup|psi|, beta and T; its verdict
// (and message) is kept per problem, so repeated calls on one problem, the
// usual case, skip the 2e5-point scan.  At most 256 problems are kept.
bool admissible(const pdd_branching_problem& B, std::string* why) {
  std::array<double, 8> key;
  for (int k = 0; k < 5; ++k) key[k] = B.alpha[k];
  key[5] = B.psi_sup;
  key[6] = B.beta;
  key[7] = B.T;
  std::string k_bytes(reinterpret_cast<const char*>(key.data()), sizeof(key));
  static std::mutex mu;
  static std::unordered_map<std::string, std::pair<bool, std::string>> seen;
  {
    std::lock_guard<std::mutex> lock(mu);
    auto it = seen.find(k_bytes);
    if (it != seen.end()) {
      if (why) *why = it->second.second;
      return it->second.first;
    }
  }
  std::string msg;
  const bool ok = admissible_scan(B, &msg);
  std::lock_guard<std::mutex> lock(mu);
  if (seen.size() >= 256) seen.clear();
  seen.emplace(std::move(k_bytes), std::make_pair(ok, msg));
  if (why) *why = msg;
  return ok;
}

// Branching problem checks shared by pdd_branching_eval and pdd_branching_bvp.
pdd_status check_branching(const pdd_branching_problem& B, const pdd_options& o, int64_t trees, int64_t n_points) {
  if (B.dim < 1 || B.dim > 3) return fail(PDD_ERR_INVALID_ARG, "dim must be 1..3");
  if (!(B.sigma >= 0.0) || !std::isfinite(B.sigma)) return fail(PDD_ERR_INVALID_ARG, "sigma must be >= 0");
  if (!(B.beta > 0.0) || !std::isfinite(B.beta)) return fail(PDD_ERR_INVALID_ARG, "beta must be positive");
  if (!(B.T >= 0.0) || !std::isfinite(B.T)) return fail(PDD_ERR_INVALID_ARG, "T must be >= 0");
  if (B.max_segments < 1 || B.max_segments > 4096) return fail(PDD_ERR_INVALID_ARG, "max_segments must be 1..4096");
  double qs = 0.0;
  for (int k = 0; k < 5; ++k) {
    if (!(B.q[k] >= 0.0) || !std::isfinite(B.alpha[k])) return fail(PDD_ERR_INVALID_ARG, "q must be >= 0, alpha finite");
    if (B.alpha[k] != 0.0 && !(B.q[k] > 0.0)) return fail(PDD_ERR_INVALID_ARG, "q_i must be > 0 where alpha_i != 0");
    qs += B.q[k];
  }
  if (std::fabs(qs - 1.0) > 1e-12) return fail(PDD_ERR_INVALID_ARG, "q must sum to 1");
  if (!(B.psi_sup > 0.0) || !std::isfinite(B.psi_sup)) return fail(PDD_ERR_INVALID_ARG, "psi_sup must be positive");
  if (trees < 0 || trees > (int64_t)0x7FFFFFFF) return fail(PDD_ERR_INVALID_ARG, "trees_per_point must be in [0, 2^31)");
  if (n_points < 0 || n_points > (int64_t)1 << 30) return fail(PDD_ERR_INVALID_ARG, "n_points out of range");
  if (o.precision < PDD_FP64_PLAIN || o.precision > PDD_FP32_STEP) return fail(PDD_ERR_INVALID_ARG, "unknown precision");
  if (o.rng_layout != PDD_RNG_PAIR52 && o.rng_layout != PDD_RNG_QUAD24) return fail(PDD_ERR_INVALID_ARG, "unknown rng layout");
  if (o.precision == PDD_FP32_STEP && o.rng_layout != PDD_RNG_QUAD24)
    return fail(PDD_ERR_INVALID_ARG, "FP32 positions require the QUAD24 layout");
  if (o.dump_steps && !o.dump_phi) return fail(PDD_ERR_INVALID_ARG, "dump_steps needs dump_phi");
  if (o.boundary_correction < 0 || o.boundary_correction > 1)
    return fail(PDD_ERR_INVALID_ARG, "boundary_correction must be 0 or 1");
  return check_fun(B.psi, B.dim, "psi", kMaxTerms, kMaxPolyG);
}

void fill_branch_params(const pdd_branching_problem& B, uint64_t seed, Tables& T, BranchParams& bp) {
  bp.dim = B.dim;
  bp.max_segments = B.max_segments;
  int L = 0;
  for (int k = 0; k < 5; ++k)
    if (B.q[k] > 0.0) L = k;
  bp.label_base = std::max(2, L);
  bp.sigma = B.sigma;
  bp.beta = B.beta;
  bp.T = B.T;
  bp.sigmaf = (float)B.sigma;
  bp.betaf = (float)B.beta;
  bp.Tf = (float)B.T;
  double cum = 0.0;
  for (int k = 0; k < 5; ++k) {
    bp.alpha[k] = B.alpha[k];
    bp.q[k] = B.q[k];
    bp.ratio[k] = B.q[k] > 0.0 ? B.alpha[k] / B.q[k] : 0.0;
    cum += B.q[k];
    bp.qcum[k] = cum;
    bp.qcumf[k] = (float)cum;
  }
  bp.inv_betaf = (float)(1.0 / B.beta);
  // compact offspring law: classes with q > 0, their cumulative thresholds
  bp.n_cls = 0;
  for (int k = 0; k < 5; ++k)
    if (B.q[k] > 0.0) {
      bp.cls[bp.n_cls] = k;
      bp.mark[bp.n_cls] = bp.ratio[k];
      ++bp.n_cls;
    }
  for (int j = 0; j < 4; ++j) {
    const bool real = j < bp.n_cls - 1;
    bp.thr[j] = real ? bp.qcum[bp.cls[j]] : INFINITY;
    bp.thrf[j] = real ? bp.qcumf[bp.cls[j]] : INFINITY;
  }
  for (int j = bp.n_cls; j < 5; ++j) {
    bp.cls[j] = bp.cls[bp.n_cls - 1];
    bp.mark[j] = bp.mark[bp.n_cls - 1];
  }
  bp.key0 = (uint32_t)seed;
  bp.key1 = (uint32_t)(seed >> 32);
  bp.psi = T.add(B.psi, B.dim, 0, true);
  bp.n_fac = (int)T.fac.size();
}

// Problem-specialised branching kernel when psi (or g) has generic terms,
// under options.specialize as for the walks: 0 = compile at run time and fall
// back to the table-driven kernel (with a note on stderr), 1 = required, -1 =
// never.  *fn stays null when the table-driven kernel is to be used.
pdd_status branch_spec(const pdd_options& o, const BranchParams& bp, const DevFun* g, const Tables& T, bool fp32,
                       int dim, bool boundary, hipFunction_t* fn) {
  *fn = nullptr;
  const bool terms = bp.psi.n_terms > 0 || (g != nullptr && g->n_terms > 0);
  if (!terms || o.specialize < 0) return PDD_OK;
  const std::string src = spec_psi_source(bp.psi, g, T.fac);
  std::string why = "a scale or shift is not finite";
  if (src.empty() ||
      !spec_branch_kernel(src, fp32, dim, fp32 ? (int)PDD_RNG_QUAD24 : o.rng_layout, boundary, fn, &why)) {
    *fn = nullptr;
    if (o.specialize == 1) return fail(PDD_ERR_HIP, "problem-specialised kernel: " + why);
    static std::once_flag once;
    std::call_once(once, [&] {
      std::fprintf(stderr, "pdd: problem-specialised branching kernel unavailable, using the table-driven kernel: %s\n",
                   why.c_str());
    });
  }
  return PDD_OK;
}

pdd_status run_branching(const pdd_branching_problem* Bp, const double* points, int64_t n_points, int64_t trees,
                         uint64_t seed, const pdd_options* op, pdd_node_stat* out, hipStream_t st) {
  if (Bp == nullptr || op == nullptr) return fail(PDD_ERR_INVALID_ARG, "problem or options is NULL");
  const pdd_branching_problem& B = *Bp;
  const pdd_options& o = *op;
  pdd_status s;
  if ((s = check_branching(B, o, trees, n_points)) != PDD_OK) return s;
  std::string why;
  if (!admissible(B, &why)) return fail(PDD_ERR_NOT_ADMISSIBLE, why);
  if (n_points > 0) {
    if ((s = check_device_ptr(points, "points_dev")) != PDD_OK) return s;
    if ((s = check_device_ptr(out, "out_dev")) != PDD_OK) return s;
  }
  if (n_points == 0) return PDD_OK;
  const bool fp32 = o.precision == PDD_FP32_STEP;

  std::unique_ptr<Plan> plan(new Plan());
  Plan& pl = *plan;
  pl.branch = true;
  PDD_HIP(hipGetDevice(&pl.device));
  if ((s = counters(&pl.ctr)) != PDD_OK) return s;
  Tables T;
  BranchParams& bp = pl.bp;
  fill_branch_params(B, seed, T, bp);
  hipFunction_t spec = nullptr;
  if ((s = branch_spec(o, bp, nullptr, T, fp32, B.dim, false, &spec)) != PDD_OK) return s;
  const Tuning tune = choose_schedule(PDD_KERNEL_BRANCH, B.dim, fp32 ? PDD_FP32_STEP : PDD_FP64, o, device_cus(),
                                      n_points * trees);
  Items items = make_items(n_points, nullptr, trees, tune.chunk_paths, {});
  const int n_items = (int)items.q.size();
  const int max_blocks = tune.blocks_per_cu * device_cus();
  const int need = (n_items + kBlock / kWave - 1) / (kBlock / kWave);
  const int grid = std::max(1, std::min(max_blocks, need));
  const int64_t spill_entries = std::max(0, B.max_segments - branch_lds_depth(fp32));

  Arena A;
  const size_t o_call = add_call_block(A, T.jobs.size());
  const size_t o_perm = A.add(sizeof(int32_t) * std::max<size_t>(1, T.perm.size()));
  const size_t o_fac = A.add(sizeof(DevFactor) * std::max<size_t>(1, T.fac.size()));
  const size_t o_cd = A.add(sizeof(double) * std::max(1, T.ncoef));
  const size_t o_cf = A.add(sizeof(float) * std::max(1, T.ncoef));
  const size_t o_q = A.add(sizeof(uint32_t) * 4);
  const size_t o_items = A.add(sizeof(WorkItem) * std::max(1, n_items));
  const size_t o_istat = A.add(sizeof(ItemStat) * std::max(1, n_items));
  const size_t o_first = A.add(sizeof(int64_t) * ((size_t)n_points + 1));
  const size_t o_spill =
      A.add(branch_stack_entry_bytes(fp32) * (size_t)std::max<int64_t>(1, spill_entries) * (size_t)grid * kBlock);
  ArenaLease lease;
  PDD_HIP(lease_arena(A.total, st, &lease, &pl.arena));
  char* base = (char*)pl.arena;
  pl.d_call = (CallPtrs*)(base + o_call);
  pl.d_jobs = (StageJob*)(base + o_call + kJobsOff);
  pl.n_jobs = (int)T.jobs.size();
  pl.d_perm = (int32_t*)(base + o_perm);
  pl.d_cd = (double*)(base + o_cd);
  pl.d_cf = (float*)(base + o_cf);
  pl.d_qhead = (uint32_t*)(base + o_q);
  pl.d_istat = (ItemStat*)(base + o_istat);
  pl.d_first = (int64_t*)(base + o_first);
  pl.n_nodes = n_points;
  pl.has_out = true;
  bp.fac = (const DevFactor*)(base + o_fac);
  bp.cd = pl.d_cd;
  bp.cf = pl.d_cf;
  bp.points = points;
  std::vector<Upload> ups;
  CallPtrs cpb{};
  cpb.out = out;
  put(ups, o_call, call_block_image(cpb, T.jobs));
  put(ups, o_perm, T.perm);
  put(ups, o_fac, T.fac);
  put(ups, o_first, items.first);
  put(ups, o_items, items.q);
  for (const auto& u : ups)
    if (!u.bytes.empty()) PDD_HIP(hipMemcpyAsync(base + u.off, u.bytes.data(), u.bytes.size(), hipMemcpyHostToDevice, st));
  BranchLaunch& BL = pl.bl;
  BL.P = &pl.bp;
  BL.fp32 = fp32;
  BL.layout = o.rng_layout;
  BL.grid = grid;
  BL.items = (const WorkItem*)(base + o_items);
  BL.n_items = n_items;
  BL.qhead = pl.d_qhead;
  BL.istat = pl.d_istat;
  BL.dump_val = o.dump_phi;
  BL.dump_segs = o.dump_steps;
  BL.trees = trees;
  BL.stack = base + o_spill;
  BL.stack_entries = spill_entries;
  BL.spec = spec;
  hipError_t e = pl.enqueue(st);
  (void)lease.done();
  if (e != hipSuccess) return fail(PDD_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
  return PDD_OK;
}

pdd_status run_branching_bvp(const pdd_branching_problem* Bp, const pdd_branching_boundary* Dp, const double* points,
                             int64_t n_points, int64_t trees, uint64_t seed, const pdd_options* op, pdd_node_stat* out,
                             hipStream_t st) {
  if (Bp == nullptr || Dp == nullptr || op == nullptr)
    return fail(PDD_ERR_INVALID_ARG, "problem, boundary or options is NULL");
  const pdd_branching_problem& B = *Bp;
  const pdd_branching_boundary& Bd = *Dp;
  const pdd_options& o = *op;
  pdd_status s;
  if ((s = check_branching(B, o, trees, n_points)) != PDD_OK) return s;
  const pdd_domain& D = Bd.domain;
  if (D.kind != PDD_DOM_BOX && D.kind != PDD_DOM_BALL && D.kind != PDD_DOM_FREE)
    return fail(PDD_ERR_INVALID_ARG, "unknown domain kind");
  if (D.kind != PDD_DOM_FREE) {
    if (D.dim != B.dim) return fail(PDD_ERR_INVALID_ARG, "boundary domain dim differs from the problem's");
    if (D.kind == PDD_DOM_BOX)
      for (int k = 0; k < D.dim; ++k)
        if (!(D.lo[k] < D.hi[k]) || !std::isfinite(D.lo[k]) || !std::isfinite(D.hi[k]))
          return fail(PDD_ERR_INVALID_ARG, "box needs finite lo < hi");
    if (D.kind == PDD_DOM_BALL && !(D.radius > 0.0 && std::isfinite(D.radius)))
      return fail(PDD_ERR_INVALID_ARG, "ball radius must be positive");
  }
  // g reads coordinates 0..dim-1 and the time argument as coordinate dim
  if ((s = check_fun(Bd.g, B.dim + 1, "g", kMaxTerms, kMaxPolyG)) != PDD_OK) return s;
  if (!(Bd.g_sup >= 0.0) || !std::isfinite(Bd.g_sup)) return fail(PDD_ERR_INVALID_ARG, "g_sup must be >= 0");
  if (!(Bd.dt > 0.0) || !std::isfinite(Bd.dt)) return fail(PDD_ERR_INVALID_ARG, "dt must be positive");
  if (Bd.n_times < 1 || Bd.n_times > kMaxTimes)
    return fail(PDD_ERR_UNSUPPORTED, "n_times must be 1.." + std::to_string(kMaxTimes));
  if (Bd.times == nullptr) return fail(PDD_ERR_INVALID_ARG, "times_host is NULL");
  for (int i = 0; i < Bd.n_times; ++i)
    if (!(Bd.times[i] >= 0.0) || !std::isfinite(Bd.times[i]) || (i > 0 && !(Bd.times[i] > Bd.times[i - 1])))
      return fail(PDD_ERR_INVALID_ARG, "times must be finite, >= 0 and increasing");
  const double tlast = Bd.times[Bd.n_times - 1];
  const double per = o.precision == PDD_FP32_STEP || o.rng_layout == PDD_RNG_QUAD24 ? 4.0 : 2.0;
  if ((std::ceil(tlast / Bd.dt) + Bd.n_times + 2.0) * B.dim / per >= 65536.0)
    return fail(PDD_ERR_UNSUPPORTED, "more than 2^16 Gaussian blocks per particle: raise dt");
  if (n_points >= ((int64_t)1 << 24)) return fail(PDD_ERR_UNSUPPORTED, "n_points must be below 2^24");
  pdd_branching_problem Ba = B;   // admissibility over [0, t_last] with sup |psi| and sup |g|
  Ba.T = tlast;
  Ba.psi_sup = std::max(B.psi_sup, Bd.g_sup);
  std::string why;
  if (!admissible(Ba, &why)) return fail(PDD_ERR_NOT_ADMISSIBLE, why);
  if (n_points > 0) {
    if ((s = check_device_ptr(points, "points_dev")) != PDD_OK) return s;
    if ((s = check_device_ptr(out, "out_dev")) != PDD_OK) return s;
  }
  if (n_points == 0) return PDD_OK;
  const bool fp32 = o.precision == PDD_FP32_STEP;

  std::unique_ptr<Plan> plan(new Plan());
  Plan& pl = *plan;
  pl.branch = true;
  pl.bvp = true;
  pl.n_times = Bd.n_times;
  PDD_HIP(hipGetDevice(&pl.device));
  if ((s = counters(&pl.ctr)) != PDD_OK) return s;
  Tables T;
  BranchParams& bp = pl.bp;
  fill_branch_params(Ba, seed, T, bp);
  BranchBoundary& bb = pl.bb;
  bb.dom_kind = D.kind;
  bb.n_times = Bd.n_times;
  for (int k = 0; k < 3; ++k) {
    bb.lo[k] = D.lo[k]; bb.hi[k] = D.hi[k]; bb.ctr[k] = D.center[k];
    bb.lof[k] = (float)D.lo[k]; bb.hif[k] = (float)D.hi[k]; bb.ctrf[k] = (float)D.center[k];
  }
  bb.rad = D.radius;
  bb.rad2 = D.radius * D.radius;
  bb.radf = (float)bb.rad;
  bb.rad2f = (float)bb.rad2;
  bb.dt = Bd.dt;
  bb.dtf = (float)Bd.dt;
  // boundary correction per sub-step (c0 = -zeta(1/2)/sqrt(2 pi), as for the walk)
  bb.shift = o.boundary_correction ? 1.4603545088095868 / std::sqrt(2.0 * M_PI) : 0.0;
  bb.shiftf = (float)bb.shift;
  for (int i = 0; i < kMaxTimes; ++i) {
    bb.times[i] = i < Bd.n_times ? Bd.times[i] : tlast;
    bb.timesf[i] = (float)bb.times[i];
  }
  bb.g = T.add(Bd.g, B.dim, 0, true);
  bp.n_fac = (int)T.fac.size();
  hipFunction_t spec = nullptr;
  if ((s = branch_spec(o, bp, &bb.g, T, fp32, B.dim, true, &spec)) != PDD_OK) return s;

  const Tuning tune = choose_schedule(PDD_KERNEL_BRANCH_BVP, B.dim, fp32 ? PDD_FP32_STEP : PDD_FP64, o,
                                      device_cus(), n_points * trees);
  Items items = make_items(n_points, nullptr, trees, tune.chunk_paths, {});
  const int n_items = (int)items.q.size();
  const int max_blocks = tune.blocks_per_cu * device_cus();
  const int need = (n_items + kBlock / kWave - 1) / (kBlock / kWave);
  const int grid = std::max(1, std::min(max_blocks, need));
  const int64_t spill_entries = std::max(0, B.max_segments - branch_lds_depth(fp32));

  Arena A;
  const size_t o_call = add_call_block(A, T.jobs.size());
  const size_t o_perm = A.add(sizeof(int32_t) * std::max<size_t>(1, T.perm.size()));
  const size_t o_fac = A.add(sizeof(DevFactor) * std::max<size_t>(1, T.fac.size()));
  const size_t o_cd = A.add(sizeof(double) * std::max(1, T.ncoef));
  const size_t o_cf = A.add(sizeof(float) * std::max(1, T.ncoef));
  const size_t o_q = A.add(sizeof(uint32_t) * 4);
  const size_t o_items = A.add(sizeof(WorkItem) * std::max(1, n_items));
  const size_t o_istat = A.add(sizeof(ItemStat) * (size_t)std::max(1, n_items) * (size_t)Bd.n_times);
  const size_t o_first = A.add(sizeof(int64_t) * ((size_t)n_points + 1));
  const size_t o_spill =
      A.add(branch_stack_entry_bytes(fp32) * (size_t)std::max<int64_t>(1, spill_entries) * (size_t)grid * kBlock);
  ArenaLease lease;
  PDD_HIP(lease_arena(A.total, st, &lease, &pl.arena));
  char* base = (char*)pl.arena;
  pl.d_call = (CallPtrs*)(base + o_call);
  pl.d_jobs = (StageJob*)(base + o_call + kJobsOff);
  pl.n_jobs = (int)T.jobs.size();
  pl.d_perm = (int32_t*)(base + o_perm);
  pl.d_cd = (double*)(base + o_cd);
  pl.d_cf = (float*)(base + o_cf);
  pl.d_qhead = (uint32_t*)(base + o_q);
  pl.d_istat = (ItemStat*)(base + o_istat);
  pl.d_first = (int64_t*)(base + o_first);
  pl.n_nodes = n_points;
  pl.n_items = n_items;
  pl.has_out = true;
  bp.fac = (const DevFactor*)(base + o_fac);
  bp.cd = pl.d_cd;
  bp.cf = pl.d_cf;
  bp.points = points;
  std::vector<Upload> ups;
  CallPtrs cpb{};
  cpb.out = out;
  put(ups, o_call, call_block_image(cpb, T.jobs));
  put(ups, o_perm, T.perm);
  put(ups, o_fac, T.fac);
  put(ups, o_first, items.first);
  put(ups, o_items, items.q);
  for (const auto& u : ups)
    if (!u.bytes.empty()) PDD_HIP(hipMemcpyAsync(base + u.off, u.bytes.data(), u.bytes.size(), hipMemcpyHostToDevice, st));
  BranchBvpLaunch& L = pl.bvl;
  L.P = &pl.bp;
  L.B = &pl.bb;
  L.fp32 = fp32;
  L.layout = o.rng_layout;
  L.grid = grid;
  L.items = (const WorkItem*)(base + o_items);
  L.n_items = n_items;
  L.qhead = pl.d_qhead;
  L.istat = pl.d_istat;
  L.dump_val = o.dump_phi;
  L.dump_segs = o.dump_steps;
  L.trees = trees;
  L.stack = base + o_spill;
  L.stack_entries = spill_entries;
  L.spec = spec;
  hipError_t e = pl.enqueue(st);
  (void)lease.done();
  if (e != hipSuccess) return fail(PDD_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
  return PDD_OK;
}

}  // namespace

// ============================================================================= C ABI
extern "C" {

pdd_status pdd_mc_interface(const pdd_linear_problem* problem, const double* nodes_dev, int64_t n_nodes,
                            const int64_t* paths_host, double dt, uint64_t seed, const pdd_options* options,
                            pdd_node_stat* out_dev, void* hip_stream) {
  try {
    if (options == nullptr) return fail(PDD_ERR_INVALID_ARG, "options is NULL");
    LinearPlanArgs a{problem, nodes_dev, n_nodes, paths_host, dt, seed, *options, out_dev, false, nullptr, nullptr,
                     nullptr, 0};
    return run_linear(a, (hipStream_t)hip_stream);
  } catch (const std::bad_alloc&) {
    return fail(PDD_ERR_NO_MEMORY, "host allocation failed");
  } catch (...) {
    return fail(PDD_ERR_HIP, "unexpected exception");
  }
}

pdd_status pdd_mc_interface_batch(const pdd_linear_problem* problems, int32_t n_problems,
                                  const int32_t* node_problem_host, const double* nodes_dev, int64_t n_nodes,
                                  const int64_t* paths_host, double dt, uint64_t seed, const pdd_options* options,
                                  pdd_node_stat* out_dev, void* hip_stream) {
  try {
    if (options == nullptr) return fail(PDD_ERR_INVALID_ARG, "options is NULL");
    BatchArgs a{problems, n_problems, node_problem_host, nodes_dev, n_nodes, paths_host, dt, seed, *options,
                out_dev, false};
    return run_linear_batch(a, (hipStream_t)hip_stream);
  } catch (const std::bad_alloc&) {
    return fail(PDD_ERR_NO_MEMORY, "host allocation failed");
  } catch (...) {
    return fail(PDD_ERR_HIP, "unexpected exception");
  }
}

pdd_status pdd_wos_interface_batch(const pdd_linear_problem* problems, int32_t n_problems,
                                   const int32_t* node_problem_host, const double* nodes_dev, int64_t n_nodes,
                                   const int64_t* paths_host, double eps, uint64_t seed, const pdd_options* options,
                                   pdd_node_stat* out_dev, void* hip_stream) {
  try {
    if (options == nullptr) return fail(PDD_ERR_INVALID_ARG, "options is NULL");
    BatchArgs a{problems, n_problems, node_problem_host, nodes_dev, n_nodes, paths_host, eps, seed, *options,
                out_dev, true};
    return run_linear_batch(a, (hipStream_t)hip_stream);
  } catch (const std::bad_alloc&) {
    return fail(PDD_ERR_NO_MEMORY, "host allocation failed");
  } catch (...) {
    return fail(PDD_ERR_HIP, "unexpected exception");
  }
}

pdd_status pdd_wos_interface(const pdd_linear_problem* problem, const double* nodes_dev, int64_t n_nodes,
                             const int64_t* paths_host, double eps, uint64_t seed, const pdd_options* options,
                             pdd_node_stat* out_dev, void* hip_stream) {
  try {
    if (options == nullptr) return fail(PDD_ERR_INVALID_ARG, "options is NULL");
    LinearPlanArgs a{problem, nodes_dev, n_nodes, paths_host, eps, seed, *options, out_dev, false, nullptr, nullptr,
                     nullptr, 0};
    a.wos = true;
    return run_linear(a, (hipStream_t)hip_stream);
  } catch (const std::bad_alloc&) {
    return fail(PDD_ERR_NO_MEMORY, "host allocation failed");
  } catch (...) {
    return fail(PDD_ERR_HIP, "unexpected exception");
  }
}

pdd_status pdd_branching_bvp(const pdd_branching_problem* problem, const pdd_branching_boundary* boundary,
                             const double* points_dev, int64_t n_points, int64_t trees_per_point, uint64_t seed,
                             const pdd_options* options, pdd_node_stat* out_dev, void* hip_stream) {
  try {
    return run_branching_bvp(problem, boundary, points_dev, n_points, trees_per_point, seed, options, out_dev,
                             (hipStream_t)hip_stream);
  } catch (const std::bad_alloc&) {
    return fail(PDD_ERR_NO_MEMORY, "host allocation failed");
  } catch (...) {
    return fail(PDD_ERR_HIP, "unexpected exception");
  }
}

pdd_status pdd_branching_eval(const pdd_branching_problem* problem, const double* points_dev, int64_t n_points,
                              int64_t trees_per_point, uint64_t seed, const pdd_options* options,
                              pdd_node_stat* out_dev, void* hip_stream) {
  try {
    return run_branching(problem, points_dev, n_points, trees_per_point, seed, options, out_dev,
                         (hipStream_t)hip_stream);
  } catch (const std::bad_alloc&) {
    return fail(PDD_ERR_NO_MEMORY, "host allocation failed");
  } catch (...) {
    return fail(PDD_ERR_HIP, "unexpected exception");
  }
}

pdd_status pdd_mc_adjoint(const pdd_linear_problem* problem, const double* nodes_dev, int64_t n_nodes,
                          const int64_t* paths_host, double dt, uint64_t seed, const pdd_options* options,
                          const double* w_dev, const pdd_fun_grad* grads_host, pdd_node_stat* out_dev,
                          void* hip_stream) {
  try {
    if (options == nullptr) return fail(PDD_ERR_INVALID_ARG, "options is NULL");
    LinearPlanArgs a{problem, nodes_dev, n_nodes, paths_host, dt, seed, *options, out_dev, true, w_dev, grads_host,
                     nullptr, 0};
    return run_linear(a, (hipStream_t)hip_stream);
  } catch (const std::bad_alloc&) {
    return fail(PDD_ERR_NO_MEMORY, "host allocation failed");
  } catch (...) {
    return fail(PDD_ERR_HIP, "unexpected exception");
  }
}

pdd_status pdd_mc_value_jacobian(const pdd_linear_problem* problem, const double* nodes_dev, int64_t n_nodes,
                                 const int64_t* paths_host, double dt, uint64_t seed, const pdd_options* options,
                                 pdd_node_stat* out_dev, double* jac_dev, int64_t jac_ld, void* hip_stream) {
  try {
    if (options == nullptr) return fail(PDD_ERR_INVALID_ARG, "options is NULL");
    if (problem == nullptr) return fail(PDD_ERR_INVALID_ARG, "problem is NULL");
    if (n_nodes > 0 && jac_dev == nullptr) return fail(PDD_ERR_INVALID_ARG, "jac_dev is NULL");
    LinearPlanArgs a{problem, nodes_dev, n_nodes, paths_host, dt, seed, *options, out_dev, true, nullptr, nullptr,
                     jac_dev, jac_ld};
    return run_linear(a, (hipStream_t)hip_stream);
  } catch (const std::bad_alloc&) {
    return fail(PDD_ERR_NO_MEMORY, "host allocation failed");
  } catch (...) {
    return fail(PDD_ERR_HIP, "unexpected exception");
  }
}

int64_t pdd_param_count(const pdd_linear_problem* problem) {
  if (problem == nullptr || problem->domain.dim < 1 || problem->domain.dim > 3) return -1;
  return param_count(*problem);
}

pdd_status pdd_query_warnings(void* hip_stream, int64_t* censored_out, int64_t* redrawn_out) {
  unsigned long long* c = nullptr;
  pdd_status s = counters(&c);
  if (s != PDD_OK) return s;
  PDD_HIP(hipStreamSynchronize((hipStream_t)hip_stream));
  unsigned long long h[2] = {0, 0}, z[2] = {0, 0};
  PDD_HIP(hipMemcpy(h, c, sizeof(h), hipMemcpyDeviceToHost));
  PDD_HIP(hipMemcpy(c, z, sizeof(z), hipMemcpyHostToDevice));
  if (censored_out) *censored_out = (int64_t)h[0];
  if (redrawn_out) *redrawn_out = (int64_t)h[1];
  if (h[0] > 0) return PDD_WARN_CENSORED;
  if (h[1] > 0) return PDD_WARN_REDRAWN;
  return PDD_OK;
}

int64_t pdd_item_count(int32_t kernel, int32_t dim, int64_t n_nodes, const int64_t* paths_host,
                       const pdd_options* options) {
  try {
    if (options == nullptr) return fail(PDD_ERR_INVALID_ARG, "options is NULL");
    if (kernel != PDD_KERNEL_WALK && kernel != PDD_KERNEL_WOS && kernel != PDD_KERNEL_WALK_BATCH &&
        kernel != PDD_KERNEL_WOS_BATCH)
      return fail(PDD_ERR_INVALID_ARG, "kernel must be a forward walk kind");
    const bool batch = kernel == PDD_KERNEL_WALK_BATCH || kernel == PDD_KERNEL_WOS_BATCH;
    if (batch ? dim != 0 : (dim < 1 || dim > 3)) return fail(PDD_ERR_INVALID_ARG, "dim out of range");
    if (n_nodes < 0 || n_nodes > (int64_t)1 << 30) return fail(PDD_ERR_INVALID_ARG, "n_nodes out of range");
    if (n_nodes > 0 && paths_host == nullptr) return fail(PDD_ERR_INVALID_ARG, "paths_host is NULL");
    const pdd_options& o = *options;
    if (o.chunk_paths < 0 || o.blocks_per_cu < 0 || o.blocks_per_cu > 64 || o.refill_groups < 0 ||
        o.refill_groups > 64)
      return fail(PDD_ERR_INVALID_ARG, "schedule override out of range");
    int64_t total = 0;
    for (int64_t i = 0; i < n_nodes; ++i) {
      if (paths_host[i] < 0 || paths_host[i] > (int64_t)0x7FFFFFFF)
        return fail(PDD_ERR_INVALID_ARG, "paths per node must be in [0, 2^31)");
      total += paths_host[i];
    }
    const Tuning tune = choose_schedule(kernel, dim, o.precision == PDD_FP32_STEP ? PDD_FP32_STEP : PDD_FP64, o,
                                        device_cus(), total);
    return (int64_t)make_items(n_nodes, paths_host, 0, tune.chunk_paths, {}).q.size();
  } catch (const std::bad_alloc&) {
    return fail(PDD_ERR_NO_MEMORY, "host allocation failed");
  } catch (...) {
    return fail(PDD_ERR_HIP, "unexpected exception");
  }
}

pdd_status pdd_set_schedule(int32_t kernel, int32_t dim, int32_t precision, const pdd_launch_schedule* s) {
  try {
    if (!schedule_kind_valid(kernel, dim, precision)) return fail(PDD_ERR_INVALID_ARG, "unknown schedule key");
    if (set_schedule(kernel, dim, precision, s) != 0) return fail(PDD_ERR_INVALID_ARG, "schedule out of range");
    return PDD_OK;
  } catch (...) {
    return fail(PDD_ERR_HIP, "unexpected exception");
  }
}

pdd_status pdd_get_schedule(int32_t kernel, int32_t dim, int32_t precision, pdd_launch_schedule* out, int32_t* tuned) {
  try {
    if (!schedule_kind_valid(kernel, dim, precision)) return fail(PDD_ERR_INVALID_ARG, "unknown schedule key");
    if (out == nullptr) return fail(PDD_ERR_INVALID_ARG, "out is NULL");
    get_schedule(kernel, dim, precision, out, tuned);
    return PDD_OK;
  } catch (...) {
    return fail(PDD_ERR_HIP, "unexpected exception");
  }
}

pdd_status pdd_save_schedules(const char* path) {
  try {
    if (save_schedules(path) != 0) return fail(PDD_ERR_INVALID_ARG, "cannot write the schedule file");
    return PDD_OK;
  } catch (...) {
    return fail(PDD_ERR_HIP, "unexpected exception");
  }
}

pdd_status pdd_load_schedules(const char* path) {
  try {
    if (load_schedules(path) < 0) return fail(PDD_ERR_INVALID_ARG, "cannot read the schedule file");
    return PDD_OK;
  } catch (...) {
    return fail(PDD_ERR_HIP, "unexpected exception");
  }
}

pdd_status pdd_release_workspace(void) {
  PDD_HIP(hipDeviceSynchronize());
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_plans.clear();
  }
  PDD_HIP(release_stream_arenas());
  PDD_HIP(trim_pools());
  return PDD_OK;
}

int64_t pdd_cached_plan_count(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  return (int64_t)g_plans.size();
}

pdd_status pdd_jacobian_apply(const double* jac_dev, int64_t n_nodes, int64_t jac_ld, int64_t n_params,
                              const double* w_dev, double* grad_dev, void* hip_stream) {
  try {
    if (n_nodes < 0 || n_params < 0 || jac_ld < n_params) return fail(PDD_ERR_INVALID_ARG, "bad Jacobian sizes");
    if (n_params == 0) return PDD_OK;
    pdd_status s;
    if ((s = check_device_ptr(grad_dev, "grad_dev")) != PDD_OK) return s;
    if (n_nodes > 0) {
      if ((s = check_device_ptr(jac_dev, "jac_dev")) != PDD_OK) return s;
      if ((s = check_device_ptr(w_dev, "w_dev")) != PDD_OK) return s;
    }
    PDD_HIP(launch_jacobian_apply(jac_dev, n_nodes, jac_ld, n_params, w_dev, nullptr, nullptr, grad_dev, nullptr,
                                  (hipStream_t)hip_stream));
    return PDD_OK;
  } catch (...) {
    return fail(PDD_ERR_HIP, "unexpected exception");
  }
}

pdd_status pdd_misfit_gradient(const pdd_node_stat* stats_dev, const double* data_dev, int64_t n_nodes,
                               const double* jac_dev, int64_t jac_ld, int64_t n_params, double* loss_dev,
                               double* grad_dev, void* hip_stream) {
  try {
    if (n_nodes < 0 || n_params < 0 || jac_ld < n_params) return fail(PDD_ERR_INVALID_ARG, "bad Jacobian sizes");
    pdd_status s;
    if ((s = check_device_ptr(loss_dev, "loss_dev")) != PDD_OK) return s;
    if (n_params > 0 && (s = check_device_ptr(grad_dev, "grad_dev")) != PDD_OK) return s;
    if (n_nodes > 0) {
      if ((s = check_device_ptr(stats_dev, "stats_dev")) != PDD_OK) return s;
      if ((s = check_device_ptr(data_dev, "data_dev")) != PDD_OK) return s;
      if (n_params > 0 && (s = check_device_ptr(jac_dev, "jac_dev")) != PDD_OK) return s;
    }
    PDD_HIP(launch_jacobian_apply(jac_dev, n_nodes, jac_ld, n_params, nullptr, stats_dev, data_dev,
                                  n_params > 0 ? grad_dev : nullptr, loss_dev, (hipStream_t)hip_stream));
    return PDD_OK;
  } catch (...) {
    return fail(PDD_ERR_HIP, "unexpected exception");
  }
}

pdd_status pdd_merge_estimates(pdd_node_stat* acc_dev, double* acc_jac_dev, int64_t acc_ld,
                               const pdd_node_stat* add_dev, const double* add_jac_dev, int64_t add_ld,
                               int64_t n_params, const int64_t* index_dev, int64_t n_add, void* hip_stream) {
  try {
    if (n_add < 0 || n_params < 0) return fail(PDD_ERR_INVALID_ARG, "negative size");
    if (n_add == 0) return PDD_OK;
    if ((acc_jac_dev == nullptr) != (add_jac_dev == nullptr))
      return fail(PDD_ERR_INVALID_ARG, "give both Jacobians or neither");
    if (acc_jac_dev != nullptr && (acc_ld < n_params || add_ld < n_params))
      return fail(PDD_ERR_INVALID_ARG, "Jacobian leading dimension below n_params");
    pdd_status s;
    if ((s = check_device_ptr(acc_dev, "acc_dev")) != PDD_OK) return s;
    if ((s = check_device_ptr(add_dev, "add_dev")) != PDD_OK) return s;
    if ((s = check_device_ptr(index_dev, "index_dev")) != PDD_OK) return s;
    if (acc_jac_dev != nullptr) {
      if ((s = check_device_ptr(acc_jac_dev, "acc_jac_dev")) != PDD_OK) return s;
      if ((s = check_device_ptr(add_jac_dev, "add_jac_dev")) != PDD_OK) return s;
    }
    PDD_HIP(launch_merge_estimates(acc_dev, acc_jac_dev, acc_ld, add_dev, add_jac_dev, add_ld, n_params, index_dev,
                                   n_add, (hipStream_t)hip_stream));
    return PDD_OK;
  } catch (...) {
    return fail(PDD_ERR_HIP, "unexpected exception");
  }
}

pdd_status pdd_node_moments(const pdd_node_stat* stats_dev, int64_t n_nodes, double* var_dev, double* se_dev,
                            void* hip_stream) {
  try {
    if (n_nodes < 0) return fail(PDD_ERR_INVALID_ARG, "n_nodes < 0");
    if (n_nodes == 0) return PDD_OK;
    pdd_status s;
    if ((s = check_device_ptr(stats_dev, "stats_dev")) != PDD_OK) return s;
    if (var_dev && (s = check_device_ptr(var_dev, "var_dev")) != PDD_OK) return s;
    if (se_dev && (s = check_device_ptr(se_dev, "se_dev")) != PDD_OK) return s;
    PDD_HIP(launch_node_moments(stats_dev, n_nodes, var_dev, se_dev, (hipStream_t)hip_stream));
    return PDD_OK;
  } catch (...) {
    return fail(PDD_ERR_HIP, "unexpected exception");
  }
}

const char* pdd_status_string(pdd_status status) {
  switch (status) {
    case PDD_OK: return "ok";
    case PDD_WARN_CENSORED: return "some paths were censored at max_steps";
    case PDD_WARN_REDRAWN: return "some trees were pruned and redrawn";
    case PDD_ERR_INVALID_ARG: return "invalid argument";
    case PDD_ERR_UNSUPPORTED: return "unsupported problem or option";
    case PDD_ERR_NOT_ADMISSIBLE: return "branching data not admissible (Assumption 3.2)";
    case PDD_ERR_HIP: return "HIP runtime error";
    case PDD_ERR_NO_MEMORY: return "out of memory";
  }
  return "unknown status";
}

const char* pdd_last_error(void) { return g_last_error.c_str(); }

int pdd_version(void) { return PDD_VERSION; }

}  // extern "C"
