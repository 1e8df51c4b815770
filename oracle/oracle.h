/*
 * Plain CPU FP64 oracle for the probabilistic-domain-decomposition hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP library;
 * only the test-suite, the smoke check and the benchmark's CPU-baseline leg
 * may load it.  It shares no code, header, table or constant with the HIP
 * path.
 *
 * What it computes (each function cites the passage it follows):
 *   - Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11, "Parallel random
 *     numbers: as easy as 1, 2, 3") and the two uniform lattices / Box-Muller
 *     transform used to turn its words into Gaussians;
 *   - the Feynman-Kac walk of Sec. 2.2 (eqs. 2.5-2.9) in its elliptic,
 *     pure-Dirichlet limit, with Euler-Maruyama stepping plus a boundary test
 *     (Sec. 2.1, "ingredients of PDD") and a per-node sample mean / variance
 *     (Sec. 2, the Monte Carlo estimator at each interface node);
 *   - the exact derivative of that discrete estimator with respect to the
 *     coefficients of g, f and c;
 *   - the branching-diffusion estimator of Sec. 3.1 (eq. 3.1, the particle
 *     system described after Assumption 3.1) in its marked form of Sec. 3.2,
 *     simulated per particle (depth first) and, separately, in the
 *     global-clock form of Algorithm 3.1;
 *   - the same estimator with particles stopped on a Dirichlet boundary
 *     (eq. 3.2) and evaluated at several output times of one tree
 *     (Algorithm 3.1).
 *
 * Every free choice the paper leaves open is fixed as described in the
 * project's design notes (sign of c, exit test, quadrature, RNG layout,
 * pruning/redraw rule); each one is restated at the function that makes it.
 */
#ifndef PDD_ORACLE_H
#define PDD_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_POW = 0, ORC_EXP = 1, ORC_SIN = 2, ORC_COS = 3, ORC_TANH = 4 };
enum { ORC_BOX = 0, ORC_BALL = 1, ORC_FREE = 2 };
enum { ORC_PAIR52 = 0, ORC_QUAD24 = 1 };

typedef struct {
  int32_t fn, dim, power, pad;
  double a, b;
} orc_factor;

/* F(x) = sum_t coef[t] prod_j fn(a x[dim] + b)^power  +  sum_m mono_coef[m] x^mono_exp[m] */
typedef struct {
  int32_t n_terms, n_factors;
  const orc_factor* factors;   /* [n_terms * n_factors] */
  const double* coef;          /* [n_terms] */
  int32_t n_mono, pad;
  const int32_t* mono_exp;     /* [n_mono * 3] */
  const double* mono_coef;     /* [n_mono] */
} orc_fun;

typedef struct {
  int32_t kind, dim;
  double lo[3], hi[3], center[3], radius;
} orc_domain;

/* 0.5 sigma^2 Lap u + b.grad u - c u = -f in D, u = g on dD.
 * boundary_shift = 0: the plain exit test (X outside D after a step).
 * boundary_shift = c0 > 0: the exit test of Gobet and Menozzi's boundary
 * correction for stopped Euler schemes: the path stops once X leaves D shrunk
 * by c0 sigma sqrt(dt) (ball: radius R - c0 sigma sqrt(dt); box: every face
 * moved inward by it); the exit value still uses the projection onto dD. */
typedef struct {
  orc_domain dom;
  double sigma;
  orc_fun b[3], c, f, g;
  double boundary_shift;
} orc_linear;

/* u_t = 0.5 sigma^2 Lap u + beta (sum_i alpha_i u^i - u), u(.,0) = psi, at time T */
typedef struct {
  int32_t dim, max_segments;
  double sigma, beta, T;
  double alpha[5], q[5];
  orc_fun psi;
} orc_branching;

/* Dirichlet boundary and output times of the branching estimator (eq. 3.2,
 * Algorithm 3.1).  g(x, s) is evaluated at (x_0, .., x_{dim-1}, s): a factor
 * with coordinate index dim reads the time argument s.  FREE: no boundary. */
typedef struct {
  orc_domain dom;
  orc_fun g;
  double dt;                   /* step of the boundary test */
  int32_t n_times, pad;
  const double* times;         /* [n_times], increasing, >= 0; the last is the horizon */
  double boundary_shift;       /* 0: plain test; c0 > 0: after a sub-step of length h the
                                  test uses the domain shrunk by c0 sigma sqrt(h) (Gobet and
                                  Menozzi's correction, as for the walk) */
} orc_branch_boundary;

typedef struct {
  double mean, m2;
  int64_t n, steps, censored;
} orc_stat;

/* ---- random numbers ---- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_walk_normal(uint64_t seed, int layout, uint32_t node, uint32_t path, uint64_t j);
double orc_u_quad24(uint32_t w);
double orc_u_pair52(uint32_t whi, uint32_t wlo);

/* ---- functions / domain ---- */
double orc_fun_eval(const orc_fun* F, const double* x);
int orc_inside(const orc_domain* D, const double* x);
void orc_project(const orc_domain* D, const double* x, double* out);

/* ---- linear walk (Sec. 2.2) ---- */
int orc_walk(const orc_linear* P, const double* nodes, int64_t n_nodes, const int64_t* paths,
             double dt, uint64_t seed, int layout, int64_t max_steps, int n_threads,
             orc_stat* out, double* dump_phi, int64_t* dump_steps, const int64_t* node_ids);

/* ---- Walk on Spheres (the method the paper recommends for Laplace's
   equation with Dirichlet data, Sec. 2.1): b = c = f = 0, any sigma.
   Jump n of path p moves X by r_n theta_n, r_n = dist(X, boundary of D),
   theta_n = zeta / |zeta| with zeta the walk Gaussians nd .. nd+d-1 of the
   path (same counters as orc_walk); it stops at the first r < eps (before
   jumping) with phi = g(P(X)); steps = number of jumps.  A path reaching
   max_steps jumps is censored with phi = g(P(X)).  A node outside D gives
   phi = g(P(node)), 0 jumps.  node_ids as for orc_walk.  Returns -1 if b, c or
   f is not zero. */
int orc_wos(const orc_linear* P, const double* nodes, int64_t n_nodes, const int64_t* paths,
            double eps, uint64_t seed, int layout, int64_t max_steps, int n_threads,
            orc_stat* out, double* dump_phi, int64_t* dump_steps, const int64_t* node_ids);

/* gradient of sum_i w_i * mean_i with respect to the coefficient arrays
   (accumulated into caller-zeroed arrays; NULL pointers are skipped) */
int orc_walk_adjoint(const orc_linear* P, const double* nodes, int64_t n_nodes, const int64_t* paths,
                     double dt, uint64_t seed, int layout, int64_t max_steps, int n_threads,
                     const double* w,
                     double* dg_coef, double* dg_mono, double* df_coef, double* df_mono,
                     double* dc_coef, double* dc_mono, orc_stat* out);

/* per-node Jacobian of the sample mean with respect to the coefficient
   arrays, with the spread of the per-path derivatives: for node i and
   parameter k (columns [g coef | g mono | f coef | f mono | c coef | c mono]),
   the Welford mean and sum of squared deviations over the node's paths of
   d phi_p / d theta_k.  jac_mean and jac_m2 are [n_nodes][n_params]
   (n_params = all coefficients of g, f and c); node_ids as for orc_walk. */
int orc_walk_jacobian(const orc_linear* P, const double* nodes, int64_t n_nodes, const int64_t* paths,
                      double dt, uint64_t seed, int layout, int64_t max_steps, int n_threads,
                      double* jac_mean, double* jac_m2, orc_stat* out, const int64_t* node_ids);

/* ---- branching (Sec. 3.1-3.2) ---- */
int orc_branching_dfs(const orc_branching* B, const double* points, int64_t n_points,
                      int64_t trees, uint64_t seed, int layout, int n_threads,
                      orc_stat* out, double* dump_val, int64_t* dump_segs, int64_t* redrawn);

int orc_branching_alg31(const orc_branching* B, const double* points, int64_t n_points,
                        int64_t trees, uint64_t seed, int max_particles, int n_threads,
                        orc_stat* out, int64_t* redrawn);

/* branching with a Dirichlet boundary, evaluated at every output time of one
   simulated tree: out[k * n_points + i] is the statistic of point i at time
   times[k] (its steps = particle sub-steps of all draws of the point's trees,
   the same for every k); dump_val[(i * trees + t) * n_times + k],
   dump_segs[i * trees + t] (particles of the accepted draw).
   Returns -1 on invalid arguments (including more than 2^16 Gaussian blocks
   per particle, or 2^24 points or more). */
int orc_branching_bvp(const orc_branching* B, const orc_branch_boundary* Bd, const double* points,
                      int64_t n_points, int64_t trees, uint64_t seed, int layout, int n_threads,
                      orc_stat* out, double* dump_val, int64_t* dump_segs, int64_t* redrawn);

#ifdef __cplusplus
}
#endif
#endif
