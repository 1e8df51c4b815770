/*
 * pdd.h -- C ABI of the MI355X (gfx950) library for the Monte Carlo hot path of
 * Probabilistic Domain Decomposition (Bernal, dos Reis, Smith, arXiv 1705.03666).
 *
 * Two estimators are exposed:
 *
 *  1. The value of a linear elliptic Dirichlet problem at interface nodes
 *     (Sec. 2.2, eqs. 2.3-2.9, elliptic and pure-Dirichlet limit):
 *
 *        0.5 sigma^2 Lap u + b . grad u - c u = -f   in D,     u = g on dD,
 *
 *     through the Feynman-Kac functional phi = g(X_tau) Y_tau + Z_tau with
 *     dX = b dt + sigma dW, dY = -c Y dt, dZ = f Y dt.  The SDE is integrated by
 *     Euler-Maruyama with a boundary test after each step and the exit point is
 *     projected onto dD (Sec. 2.1, "ingredients of PDD"); the per-node output is
 *     the sample mean and sum of squared deviations (Sec. 2, the Monte Carlo
 *     estimator at every interfacing node).  The sign of c is that of a killing
 *     rate (the paper's c is -c here).
 *
 *  2. The solution of the semilinear branching PDE (Sec. 3.1, eq. 3.1, and the
 *     marked representation of Sec. 3.2)
 *
 *        u_t = 0.5 sigma^2 Lap u + beta ( sum_{i<=4} alpha_i u^i - u ),  u(.,0) = psi,
 *
 *     at time T, by branching Brownian particles with Exp(beta) lifetimes,
 *     offspring counts drawn from q, weights alpha_I/q_I, and the product of psi
 *     over the particles alive at T.
 *
 * plus the exact gradient of sum_i w_i u_i (the linear estimator) with respect
 * to the coefficients of g, f and c, computed by re-simulating the same paths
 * from their counters (nothing per path is stored).
 *
 * Conventions (all entry points):
 *  - Host-callable; work is enqueued on `hip_stream` (a hipStream_t, NULL = the
 *    null stream) and is asynchronous.  Argument validation is synchronous:
 *    a negative status is returned before anything is enqueued and the reason
 *    is available from pdd_last_error() (per thread).
 *  - Pointers marked "device" must be device memory of the current HIP device,
 *    "host" pointers host memory.  The caller owns every pointer; the library
 *    never frees caller memory and keeps no caller pointer after the call
 *    returns, except that device arrays must stay valid until the enqueued
 *    work finishes.
 *  - Scratch memory.  A call's scratch (tables, work queue, per-item
 *    partials, branching stacks) lives in the call arena of its (device,
 *    stream): one buffer from a memory pool of the library's own, kept from
 *    one call to the next and grown (stream-ordered) when a call needs more,
 *    so a call frees nothing and does not wait for earlier work; calls on one
 *    stream use it in stream order, and calls from several host threads on
 *    one stream enqueue one at a time.  The
 *    graph schedule (PDD_SCHED_AUTO / PDD_SCHED_PERSISTENT_GRAPH) instead
 *    keeps a captured launch plan with its own scratch per (problem
 *    structure, budgets, step, seed, options, outputs requested, stream); at
 *    most 16 plans are cached, the least recently used one is dropped once
 *    its last launch has finished.  A plan does not depend on the caller's
 *    buffers (nodes, coefficient arrays, outputs, weights): they are handed
 *    to every replay.  pdd_release_workspace() frees the plans and the
 *    call arenas and returns the pool's memory.
 *  - Per-path values and step counts are a pure function of (problem, node,
 *    path index, dt, seed, precision, rng layout): independent of the
 *    schedule, the work-item size and the device.  Node statistics merge
 *    per-item partials in a fixed order, so they are bitwise reproducible for
 *    a fixed schedule on a fixed device; across schedules or devices the item
 *    boundaries move and the FP64 merges round differently (equal to about
 *    1e-13 relative).
 *  - No exception or abort crosses the ABI.
 */
#ifndef PDD_H
#define PDD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PDD_VERSION 1

typedef enum {
  PDD_OK = 0,
  PDD_WARN_CENSORED = 1,      /* some paths hit max_steps (see pdd_query_warnings) */
  PDD_WARN_REDRAWN = 2,       /* some branching trees were pruned and redrawn */
  PDD_ERR_INVALID_ARG = -1,
  PDD_ERR_UNSUPPORTED = -2,
  PDD_ERR_NOT_ADMISSIBLE = -3, /* branching data violate Assumption 3.2 */
  PDD_ERR_HIP = -4,
  PDD_ERR_NO_MEMORY = -5
} pdd_status;

/* ---------------------------------------------------------------- problem data */

typedef enum { PDD_DOM_BOX = 0, PDD_DOM_BALL = 1, PDD_DOM_FREE = 2 } pdd_domain_kind;

/* Open set D in R^dim, dim in 1..3.  BOX: lo[k] < x_k < hi[k].  BALL:
 * |x - center| < radius.  FREE: R^dim (branching only).  A point on dD counts
 * as outside. */
typedef struct {
  int32_t kind, dim;
  double lo[3], hi[3], center[3], radius;
} pdd_domain;

typedef enum { PDD_FN_POW = 0, PDD_FN_EXP = 1, PDD_FN_SIN = 2, PDD_FN_COS = 3, PDD_FN_TANH = 4 } pdd_fn;

/* One factor fn(a * x[dim] + b)^power (POW means the identity, so
 * (a x + b)^power; power 0 is the constant 1).  0 <= power <= 16. */
typedef struct {
  int32_t fn, dim, power, pad;
  double a, b;
} pdd_factor;

/* A coefficient function:
 *   F(x) = sum_{t<n_terms} coef[t] prod_{j<n_factors} factor[t*n_factors+j](x)
 *        + sum_m poly[m] x^alpha_m
 * The polynomial part is dense, in graded-lexicographic order of total degree
 * <= poly_degree (-1: none) in `dim` variables: degree by degree, and within a
 * degree the exponent tuples in decreasing lexicographic order (3-D: 1; x, y, z;
 * x^2, xy, xz, y^2, yz, z^2; x^3, ...).  It has C(poly_degree + dim, dim)
 * entries.  factors: host, read during the call.  coef, poly: device, read by
 * the enqueued work (these are the differentiable parameters).
 * Limits: n_factors <= 4; b, c, f: poly_degree <= 3, n_terms <= 16
 * (<= 4 for c and f in pdd_mc_adjoint); g, psi: poly_degree <= 8, n_terms <= 64. */
typedef struct {
  int32_t n_terms, n_factors;
  const pdd_factor* factors;
  const double* coef;
  int32_t poly_degree, pad;
  const double* poly;
} pdd_fun;

/* 0.5 sigma^2 Lap u + b . grad u - c u = -f in D, u = g on dD (eqs. 2.3-2.4 with
 * A = sigma^2 I; only b[0..dim-1] are read).  sigma > 0. */
typedef struct {
  pdd_domain domain;
  double sigma;
  pdd_fun b[3], c, f, g;
} pdd_linear_problem;

/* u_t = 0.5 sigma^2 Lap u + beta (sum_i alpha_i u^i - u), u(.,0) = psi, at time T
 * in R^dim (eq. 3.1; marked form of Sec. 3.2).  q is the sampling law of the
 * offspring count: q_i >= 0, sum q_i = 1, q_i > 0 wherever alpha_i != 0.
 * psi_sup bounds |psi| and is used for the admissibility test of Assumption 3.2.
 * A tree that needs more than max_segments particles (1..4096) is discarded and
 * redrawn (pruning, remark before Algorithm 3.1). */
typedef struct {
  int32_t dim, max_segments;
  double sigma, beta, T;
  double alpha[5], q[5];
  double psi_sup;
  pdd_fun psi;
} pdd_branching_problem;

/* Dirichlet boundary and output times of the branching estimator (eq. 3.2:
 * particles are stopped on the boundary of `domain`; Algorithm 3.1: one tree
 * is evaluated at several times T_0 < T_1 < ...).  domain: BOX or BALL of the
 * problem's dim, or FREE (no boundary: the free-space estimator at several
 * times).  g: boundary data g(x, s) at a boundary point x and time argument s;
 * a factor whose dim equals the problem's dim reads s (its polynomial part is
 * in x only).  g_sup bounds |g| (admissibility, with psi_sup, over
 * [0, last time]).  dt: the particles move by exact Brownian increments over
 * sub-steps of at most dt that also end at every output time and at the
 * particle's death, and are tested against the boundary after each sub-step
 * (not the one ending at the death: children are tested at birth).  times:
 * host [n_times], 1 <= n_times <= 12, finite, >= 0, strictly increasing; the
 * last one is the horizon (problem.T is not used). */
typedef struct {
  pdd_domain domain;
  pdd_fun g;
  double g_sup;
  double dt;
  int32_t n_times, pad;
  const double* times;
} pdd_branching_boundary;

/* ---------------------------------------------------------------- options */

typedef enum {
  PDD_FP64_PLAIN = 0,  /* FP64; one launch per node, one path per thread, no refill (baseline) */
  PDD_FP64 = 1,        /* FP64 stepping, batched persistent kernel */
  PDD_FP32_STEP = 2    /* FP32 stepping and transforms, FP64 accumulation (QUAD24 only) */
} pdd_precision;

typedef enum { PDD_RNG_PAIR52 = 0, PDD_RNG_QUAD24 = 1 } pdd_rng_layout;

typedef enum {
  PDD_SCHED_AUTO = 0,             /* persistent + cached graph plan */
  PDD_SCHED_PERSISTENT = 1,       /* persistent kernel, per-call scratch */
  PDD_SCHED_PERSISTENT_GRAPH = 2  /* persistent kernel captured once into a hipGraph and replayed */
} pdd_schedule;

/* The persistent kernels, as keys of the schedule table. */
typedef enum {
  PDD_KERNEL_WALK = 0,          /* pdd_mc_interface (batched forward walk) */
  PDD_KERNEL_WALK_ADJOINT = 1,  /* pdd_mc_adjoint, pdd_mc_value_jacobian */
  PDD_KERNEL_WOS = 2,           /* pdd_wos_interface */
  PDD_KERNEL_WALK_BATCH = 3,    /* pdd_mc_interface_batch (dim 0: any mix of dimensions) */
  PDD_KERNEL_WOS_BATCH = 4,     /* pdd_wos_interface_batch */
  PDD_KERNEL_BRANCH = 5,        /* pdd_branching_eval */
  PDD_KERNEL_BRANCH_BVP = 6     /* pdd_branching_bvp */
} pdd_kernel;

/* A launch schedule: paths (trees) per large work item, persistent blocks
 * per compute unit, step groups between lane refills (walks only). */
typedef struct {
  int32_t chunk_paths, blocks_per_cu, refill_groups, pad;
} pdd_launch_schedule;

/* Partial statistics of one work item (48 bytes): the Welford triple of its
 * paths, their total steps, censored paths and redrawn trees. */
typedef struct {
  double mean, m2;
  int64_t n, steps, censored, redrawn;
} pdd_item_stat;

typedef struct {
  int32_t precision;      /* pdd_precision */
  int32_t rng_layout;     /* pdd_rng_layout; PDD_FP32_STEP requires QUAD24 */
  int64_t max_steps;      /* censoring cap per path; 0 = ceil(100/dt) */
  double* dump_phi;       /* device, optional [sum(paths)]: per-path value, node-major (every linear
                             entry point except the plain adjoint; a call with dumps is never captured
                             into a cached graph) */
  int64_t* dump_steps;    /* device, optional [sum(paths)]: per-path step (segment) count */
  int32_t schedule;       /* pdd_schedule */
  int32_t chunk_paths;    /* paths per large work item (about the last eighth of each node's paths
                             goes into items of chunk_paths/8, at least 256, queued last);
                             0 = the schedule table (tuned entry, else default) */
  int32_t blocks_per_cu;  /* persistent grid size per compute unit; 0 = the schedule table */
  int32_t refill_groups;  /* step groups between lane refills; 0 = the schedule table */
  int32_t boundary_correction; /* linear walks: 0 = plain exit test (X outside D after a step);
                                  1 = boundary-corrected test of Gobet and Menozzi (Sec. 2.1 points to
                                  their schemes): the path stops once X leaves D shrunk by
                                  c0 sigma sqrt(dt), c0 = -zeta(1/2)/sqrt(2 pi) ~ 0.5826, which removes
                                  the O(sqrt dt) overshoot bias; g is still taken at the projection of
                                  X onto the boundary of D.  pdd_branching_bvp: the test after a
                                  sub-step of length h uses the domain shrunk by c0 sigma sqrt(h).
                                  Ignored by pdd_branching_eval. */
  int32_t specialize;     /* batched linear walks (PDD_FP64, PDD_FP32_STEP) whose b, c or f have generic
                             terms, and pdd_branching_eval / pdd_branching_bvp whose psi (or g) has
                             generic terms: 0 = auto: compile, at run time, a kernel with the problem's
                             factor structure (functions, coordinates, scales, shifts, powers) written
                             in as constants, and fall back to the table-driven kernel (with a note on
                             stderr) if the runtime compiler is unavailable; 1 = required (a failed
                             compilation returns PDD_ERR_HIP); -1 = never.  Both kernels evaluate the
                             same operations in the same order.  Coefficients stay run-time data, so
                             one compiled kernel (cached in memory and in $PDD_JIT_CACHE, default
                             ~/.cache/pdd_jit) serves every coefficient value.  Ignored elsewhere. */
  /* Failure / resume (pdd_mc_interface and pdd_wos_interface with PDD_FP64 or
   * PDD_FP32_STEP; else PDD_ERR_UNSUPPORTED).  A call's paths are cut into
   * pdd_item_count() work items whose partial statistics sit in fixed
   * node-major slots and are merged in slot order, and every path is a pure
   * function of (seed, node, path index); so an item lost to a fault can be
   * recomputed alone and the merged result is bit-identical to a full run.
   *  partials: device [n_items] or NULL.  When given, the call keeps the
   *    per-item partials there: it writes the slot of every item it runs and
   *    reads the slot of every item it skips.  It is the checkpoint.
   *  skip_items: host [n_items] or NULL; nonzero = do not run this item in
   *    this call (requires `partials`; its partial is taken from there).
   * A call with either set is never captured into a cached graph. */
  const uint8_t* skip_items;
  pdd_item_stat* partials;
} pdd_options;

/* Per-node result: mean and sum of squared deviations (variance = m2/(n-1),
 * standard error = sqrt(variance/n)), path count, total steps (linear) or
 * segments (branching), and censored paths / trees. 40 bytes. */
typedef struct {
  double mean, m2;
  int64_t n, steps, censored;
} pdd_node_stat;

/* Gradient outputs for one function: dcoef[n_terms], dpoly[n_mono] (device,
 * accumulated with +=; NULL skips that part). */
typedef struct {
  double* dcoef;
  double* dpoly;
} pdd_fun_grad;

/* ---------------------------------------------------------------- entry points */

/* Monte Carlo value at interface nodes (Sec. 2.2).
 *  problem:   host struct; domain BOX or BALL.
 *  nodes_dev: device [n_nodes][domain.dim] FP64.  A node outside D gets
 *             tau = 0 and phi = g(projection of the node).
 *  paths_host: host [n_nodes] path budget per node, 0 <= paths < 2^32.
 *  dt > 0: Euler-Maruyama step.  seed: Philox key.
 *  out_dev:   device [n_nodes] pdd_node_stat.
 *  Errors: PDD_ERR_INVALID_ARG (bad sizes / domain / dt / options),
 *          PDD_ERR_UNSUPPORTED (limits above exceeded), PDD_ERR_HIP. */
pdd_status pdd_mc_interface(const pdd_linear_problem* problem, const double* nodes_dev, int64_t n_nodes,
                            const int64_t* paths_host, double dt, uint64_t seed, const pdd_options* options,
                            pdd_node_stat* out_dev, void* hip_stream);

/* pdd_mc_interface for callers that cannot allocate device memory (code
 * running under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same walk, statistics and outputs, but every scratch
 * buffer of the call (staged tables, node copy, work queue, per-item
 * partials) is carved out of one fixed area of 16 MiB that the library holds
 * on each device it runs on until the process ends; the call maps no memory,
 * calls no hipMalloc / hipFree / pool allocation and compiles nothing at run
 * time (problems with generic terms in b, c or f run on the table-driven
 * kernel, which computes the same values).  The schedule option is taken as
 * PDD_SCHED_PERSISTENT (no cached graph).  A call whose scratch does not fit
 * returns PDD_ERR_UNSUPPORTED before enqueuing anything, with the sizes in
 * pdd_last_error() (4096 nodes x 1e5 paths in FP32 take about 4 MB).
 * Every call on one device shares that device's area, whose contents are the
 * last call's: calls that overlap on one GPU (two streams, two threads) race
 * and must be serialised by the caller.  Arguments and errors otherwise as
 * pdd_mc_interface. */
pdd_status pdd_mc_interface_noalloc(const pdd_linear_problem* problem, const double* nodes_dev, int64_t n_nodes,
                                    const int64_t* paths_host, double dt, uint64_t seed,
                                    const pdd_options* options, pdd_node_stat* out_dev, void* hip_stream);

/* Walk on Spheres for Laplace's equation with Dirichlet data, the method
 * Sec. 2.1 recommends for that case: b, c and f must be identically zero
 * (no terms, no polynomial; else PDD_ERR_UNSUPPORTED); sigma does not
 * matter.  Each path jumps from X to X + r theta, r = distance from X to the
 * boundary of D, theta uniform on the unit sphere (the path's Gaussians of
 * jump n, nd .. nd+d-1, normalised: same counters as pdd_mc_interface), and
 * stops once r < eps, with phi = g(projection of X onto the boundary).
 * steps in out_dev counts jumps; a path reaching options->max_steps jumps
 * (0: 100000) is censored.  Arguments as pdd_mc_interface with eps > 0 in
 * place of dt; precision FP32_STEP or FP64 (no plain variant), no boundary
 * correction, no dumps of more than phi and steps. */
pdd_status pdd_wos_interface(const pdd_linear_problem* problem, const double* nodes_dev, int64_t n_nodes,
                             const int64_t* paths_host, double eps, uint64_t seed, const pdd_options* options,
                             pdd_node_stat* out_dev, void* hip_stream);

/* Interface values of a heterogeneous batch of linear problems in one
 * persistent launch: the nodes of every subdomain of a PDD partition (or of
 * several partitions), whose domains, dimensions, operators and boundary data
 * differ, share one work queue and one grid (the loops over interface nodes
 * and samples of Algorithm 3.1).
 *  problems: host [n_problems], 1 <= n_problems <= 64; each as for
 *    pdd_mc_interface except that b, c, f are dense polynomials only (no
 *    generic terms: PDD_ERR_UNSUPPORTED); g may have terms.  Dimensions 1..3
 *    may be mixed.
 *  node_problem_host: host [n_nodes], the problem of every node.
 *  nodes_dev: device [n_nodes][3] FP64; a node uses the first dim
 *    coordinates of its row (the rest are ignored).
 *  paths_host, dt, seed, out_dev: as pdd_mc_interface; options as
 *    pdd_mc_interface except PDD_FP64_PLAIN, skip_items and partials
 *    (PDD_ERR_UNSUPPORTED).
 * Node i draws its Gaussians with node index i (its row in this batch), so
 * its paths are those pdd_mc_interface computes for a node of index i with
 * the same problem. */
pdd_status pdd_mc_interface_batch(const pdd_linear_problem* problems, int32_t n_problems,
                                  const int32_t* node_problem_host, const double* nodes_dev, int64_t n_nodes,
                                  const int64_t* paths_host, double dt, uint64_t seed, const pdd_options* options,
                                  pdd_node_stat* out_dev, void* hip_stream);

/* Walk on Spheres over a heterogeneous batch (b, c, f zero in every problem;
 * eps as pdd_wos_interface; everything else as pdd_mc_interface_batch). */
pdd_status pdd_wos_interface_batch(const pdd_linear_problem* problems, int32_t n_problems,
                                   const int32_t* node_problem_host, const double* nodes_dev, int64_t n_nodes,
                                   const int64_t* paths_host, double eps, uint64_t seed, const pdd_options* options,
                                   pdd_node_stat* out_dev, void* hip_stream);

/* Branching estimator (Sec. 3.1-3.2) at points_dev [n_points][dim] (device,
 * FP64), trees_per_point trees each (< 2^32).  out_dev: device [n_points];
 * steps = segments simulated, censored = trees that failed 16 draws (value 0).
 * Returns PDD_ERR_NOT_ADMISSIBLE when Assumption 3.2 fails for alpha, beta,
 * psi_sup and T. */
pdd_status pdd_branching_eval(const pdd_branching_problem* problem, const double* points_dev,
                              int64_t n_points, int64_t trees_per_point, uint64_t seed,
                              const pdd_options* options, pdd_node_stat* out_dev, void* hip_stream);

/* Branching estimator with a Dirichlet boundary, evaluated at every output
 * time of one simulated tree (eq. 3.2 and Algorithm 3.1, the paper's KPP
 * setting for PDD).  For a point x and output time t the tree's value is the
 * product of psi(X_t) over the particles inside the domain at t, of
 * g(X_tau, t - tau) over those stopped on the boundary at tau <= t (projected
 * onto it), and of alpha_I / q_I over the branchings before t.
 *  out_dev: device [n_times][n_points] (time-major: one pdd_node_stat array
 *  per output time); steps = particle sub-steps simulated for the point (all
 *  draws), the same for every time; censored = trees that failed 16 draws
 *  (value 0 at every time).
 *  options->dump_phi: optional device [n_points][trees][n_times] values;
 *  options->dump_steps: optional device [n_points][trees] segment counts.
 * Limits: n_points < 2^24; at most 2^16 Gaussian blocks per particle, i.e.
 * (ceil(t_last / dt) + n_times + 2) dim / m < 2^16 (m = 4 normals per block
 * for QUAD24, 2 for PAIR52), else PDD_ERR_UNSUPPORTED.  Counter layout of the
 * particle Gaussians: stream 5 (word1 = 5 << 28 | attempt << 24 | label bits
 * 32..47 << 8 | block >> 8, word3 = point | (block & 255) << 24). */
pdd_status pdd_branching_bvp(const pdd_branching_problem* problem, const pdd_branching_boundary* boundary,
                             const double* points_dev, int64_t n_points, int64_t trees_per_point, uint64_t seed,
                             const pdd_options* options, pdd_node_stat* out_dev, void* hip_stream);

/* Gradient of sum_i w_i u_i with respect to the coefficient arrays of g, f and c
 * (the exact derivative of the discrete estimator, same paths as
 * pdd_mc_interface with the same arguments).  w_dev: device [n_nodes].
 * grads_host: host array of three pdd_fun_grad {g, f, c}; the device arrays
 * they point to are accumulated into (+=).  out_dev: optional per-node stats
 * (NULL to skip).  Limits: c and f with n_terms <= 4. */
pdd_status pdd_mc_adjoint(const pdd_linear_problem* problem, const double* nodes_dev, int64_t n_nodes,
                          const int64_t* paths_host, double dt, uint64_t seed, const pdd_options* options,
                          const double* w_dev, const pdd_fun_grad* grads_host, pdd_node_stat* out_dev,
                          void* hip_stream);

/* Value and Jacobian in one pass: the per-node statistics of pdd_mc_interface
 * and, for every node i, the derivative of its sample mean u_i with respect to
 * every coefficient of g, f and c (same paths, same derivative as
 * pdd_mc_adjoint, which equals sum_i w_i * row_i).  Lets a caller form
 * the gradient of any loss of the u_i after this single pass (e.g. J^T w with
 * w = dL/du computed from out_dev) instead of re-simulating the paths.
 *  jac_dev: device [n_nodes][jac_ld] FP64, overwritten; columns in the order
 *           g.coef[n_terms], g.poly[n_mono], f.coef, f.poly, c.coef, c.poly
 *           (pdd_param_count gives their number; jac_ld >= that count).
 *  out_dev: device [n_nodes] pdd_node_stat (required).
 *  Limits and errors as for pdd_mc_adjoint. */
pdd_status pdd_mc_value_jacobian(const pdd_linear_problem* problem, const double* nodes_dev, int64_t n_nodes,
                                 const int64_t* paths_host, double dt, uint64_t seed, const pdd_options* options,
                                 pdd_node_stat* out_dev, double* jac_dev, int64_t jac_ld, void* hip_stream);

/* Number of differentiable coefficients of g, f and c (the Jacobian width);
 * -1 if the problem is malformed. */
int64_t pdd_param_count(const pdd_linear_problem* problem);

/* grad = J^T w: grad[k] = sum_i w_i jac[i][k] for a Jacobian from
 * pdd_mc_value_jacobian, i.e. the gradient of sum_i w_i u_i with respect to the
 * coefficients (the same quantity pdd_mc_adjoint accumulates, formed without
 * re-simulating the paths).  Summed in a fixed order (bitwise reproducible).
 *  jac_dev: device [n_nodes][jac_ld] FP64; w_dev: device [n_nodes];
 *  grad_dev: device [n_params], overwritten.  n_params <= jac_ld.
 * Errors: PDD_ERR_INVALID_ARG (sizes, non-device pointers), PDD_ERR_HIP. */
pdd_status pdd_jacobian_apply(const double* jac_dev, int64_t n_nodes, int64_t jac_ld, int64_t n_params,
                              const double* w_dev, double* grad_dev, void* hip_stream);

/* Data-misfit loss of the interface values and its gradient (the loss the
 * adjoint serves: a least-squares fit of the coefficients to data at the
 * nodes): loss = sum_i (u_i - d_i)^2 with u_i = stats_dev[i].mean, and
 * grad = J^T w with w_i = 2 (u_i - d_i), the exact gradient of the loss at
 * the estimate with the same samples.
 *  stats_dev: device [n_nodes] (from pdd_mc_value_jacobian); data_dev: device
 *  [n_nodes]; jac_dev: device [n_nodes][jac_ld]; loss_dev: device, one double;
 *  grad_dev: device [n_params]; both overwritten.
 * Errors as pdd_jacobian_apply. */
pdd_status pdd_misfit_gradient(const pdd_node_stat* stats_dev, const double* data_dev, int64_t n_nodes,
                               const double* jac_dev, int64_t jac_ld, int64_t n_params, double* loss_dev,
                               double* grad_dev, void* hip_stream);

/* Refines estimates with more samples: merges a second, independent sample of
 * some nodes (for instance a call with another seed over the nodes whose
 * standard error is still above a target) into existing node statistics, so
 * that the result is the sample mean over both samples (Sec. 2.1's per-node
 * mean over N + N' paths).  For k < n_add, node i = index_dev[k] of acc_dev
 * receives add_dev[k]: Welford triples merged (Chan et al.), n, steps and
 * censored summed; with Jacobians, row i of acc_jac_dev becomes the path-count
 * weighted mean (n_i row_i + n_k add_row_k) / (n_i + n_k).
 *  acc_dev: device [*] pdd_node_stat, updated; add_dev: device [n_add];
 *  index_dev: device [n_add] int64, distinct node indices (duplicates race);
 *  acc_jac_dev / add_jac_dev: device [*][acc_ld] / [n_add][add_ld] FP64, both
 *  or neither; n_params columns are merged. */
pdd_status pdd_merge_estimates(pdd_node_stat* acc_dev, double* acc_jac_dev, int64_t acc_ld,
                               const pdd_node_stat* add_dev, const double* add_jac_dev, int64_t add_ld,
                               int64_t n_params, const int64_t* index_dev, int64_t n_add, void* hip_stream);

/* Sample variance and standard error of every node (the unbiased estimator:
 * var = m2 / (n - 1), 0 for n < 2; se = sqrt(var / n), 0 for n = 0).
 *  stats_dev: device [n_nodes]; var_dev, se_dev: device [n_nodes] or NULL. */
pdd_status pdd_node_moments(const pdd_node_stat* stats_dev, int64_t n_nodes, double* var_dev, double* se_dev,
                            void* hip_stream);

/* Synchronizes hip_stream and reports (then clears) the censored-path and
 * redrawn-tree counters of the work enqueued since the last query:
 * PDD_WARN_CENSORED / PDD_WARN_REDRAWN if non-zero, else PDD_OK. */
pdd_status pdd_query_warnings(void* hip_stream, int64_t* censored_out, int64_t* redrawn_out);

/* Number of work items (partials slots) a call of `kernel` (PDD_KERNEL_WALK,
 * PDD_KERNEL_WOS, PDD_KERNEL_WALK_BATCH or PDD_KERNEL_WOS_BATCH) in dimension
 * `dim` (0 for the batch entry points) cuts these budgets into with these
 * options on the current device (the item size depends on the schedule
 * options, the schedule table, the precision, the total path count and the
 * device's compute units).  Negative pdd_status on invalid input. */
int64_t pdd_item_count(int32_t kernel, int32_t dim, int64_t n_nodes, const int64_t* paths_host,
                       const pdd_options* options);

/* Schedule table of the current device (see the options chunk_paths,
 * blocks_per_cu, refill_groups: a call takes each knob from its options when
 * non-zero, else from the table entry of (kernel, dim, precision), else from
 * the built-in default).  Entries are kept per device kind (architecture and
 * compute-unit count); the library reads $PDD_SCHEDULE_FILE (default
 * ~/.cache/pdd/schedules.txt) on its first call.  precision: PDD_FP64 or
 * PDD_FP32_STEP; dim: 1..3, or 0 for the batch kernels.
 *  pdd_set_schedule: sets (s != NULL) or removes (s == NULL) an entry of this
 *    process's table; 1 <= chunk_paths <= 2^30, 1 <= blocks_per_cu,
 *    refill_groups <= 64, else PDD_ERR_INVALID_ARG.
 *  pdd_get_schedule: the entry a call would start from (tuned, or the
 *    default), *tuned = 1 if it is a table entry.
 *  pdd_save_schedules / pdd_load_schedules: write the table to / merge a file
 *    into it (path NULL = the default file); PDD_ERR_INVALID_ARG if the file
 *    cannot be written / read. */
pdd_status pdd_set_schedule(int32_t kernel, int32_t dim, int32_t precision, const pdd_launch_schedule* s);
pdd_status pdd_get_schedule(int32_t kernel, int32_t dim, int32_t precision, pdd_launch_schedule* out, int32_t* tuned);
pdd_status pdd_save_schedules(const char* path);
pdd_status pdd_load_schedules(const char* path);

/* Frees cached launch plans, the per-stream call arenas and their device
 * memory, and returns the memory the library's pools keep (synchronizes the
 * device; no other call may run meanwhile). */
pdd_status pdd_release_workspace(void);

/* Number of cached graph launch plans (at most 16). */
int64_t pdd_cached_plan_count(void);

const char* pdd_status_string(pdd_status status);
const char* pdd_last_error(void);
int pdd_version(void);

#ifdef __cplusplus
}
#endif
#endif
