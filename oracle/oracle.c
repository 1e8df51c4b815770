/*
 * Plain CPU FP64 oracle -- TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Written for readability: one path at a time, one step at a time, in the
 * order the method defines them.  Built with -O2 -ffp-contract=off so that
 * every product and sum is rounded separately.
 */
#include "oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11, Sec. 4 / Table 2): a 4-word counter is
 * mixed by ten rounds; each round multiplies words 0 and 2 by two fixed odd
 * constants, keeps the high and low halves of the 64-bit products, and xors
 * the high halves with the other two words and the round key.  The round key
 * starts at the user key and is bumped by two Weyl constants between rounds. */
static const uint32_t PHILOX_M0 = 0xD2511F53u, PHILOX_M1 = 0xCD9E8D57u;
static const uint32_t PHILOX_W0 = 0x9E3779B9u, PHILOX_W1 = 0xBB67AE85u;

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
    uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += PHILOX_W0;
    k1 += PHILOX_W1;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform lattices.  QUAD24: the top 23 bits k of a word give u = (2k+1) 2^-24.
 * PAIR52: 52 bits k taken from two words give u = (2k+1) 2^-53.  Both are
 * strictly inside (0, 1), so log(u) is finite. */
static double u_quad24(uint32_t w) { return (2.0 * (double)(w >> 9) + 1.0) * ldexp(1.0, -24); }
static double u_pair52(uint32_t whi, uint32_t wlo) {
  uint64_t k = ((uint64_t)whi << 20) | (uint64_t)(wlo >> 12);
  return (2.0 * (double)k + 1.0) * ldexp(1.0, -53);
}

/* Box-Muller: (u_a, u_b) -> (r cos 2 pi u_b, r sin 2 pi u_b), r = sqrt(-2 ln u_a). */
static void box_muller(double ua, double ub, double* z0, double* z1) {
  double r = sqrt(-2.0 * log(ua));
  *z0 = r * cos(2.0 * M_PI * ub);
  *z1 = r * sin(2.0 * M_PI * ub);
}

static void make_key(uint64_t seed, uint32_t key[2]) {
  key[0] = (uint32_t)seed;
  key[1] = (uint32_t)(seed >> 32);
}

/* Gaussian number j of a path's stream.  Counter layout for the linear walk:
 * word0 = low 32 bits of the block index b, word1 = (stream 0) << 24 | bits
 * 32..55 of b, word2 = path index, word3 = node index. */
static double walk_normal(const uint32_t key[2], int layout, uint32_t node, uint32_t path, uint64_t j) {
  uint32_t ctr[4], w[4];
  double z[4];
  uint64_t per_block = (layout == ORC_QUAD24) ? 4 : 2;
  uint64_t blk = j / per_block;
  ctr[0] = (uint32_t)blk;
  ctr[1] = (uint32_t)((blk >> 32) & 0xFFFFFFu);
  ctr[2] = path;
  ctr[3] = node;
  orc_philox4x32_10(ctr, key, w);
  if (layout == ORC_QUAD24) {
    box_muller(u_quad24(w[0]), u_quad24(w[1]), &z[0], &z[1]);
    box_muller(u_quad24(w[2]), u_quad24(w[3]), &z[2], &z[3]);
  } else {
    box_muller(u_pair52(w[0], w[1]), u_pair52(w[2], w[3]), &z[0], &z[1]);
  }
  return z[j % per_block];
}

double orc_u_quad24(uint32_t w) { return u_quad24(w); }
double orc_u_pair52(uint32_t whi, uint32_t wlo) { return u_pair52(whi, wlo); }

double orc_walk_normal(uint64_t seed, int layout, uint32_t node, uint32_t path, uint64_t j) {
  uint32_t key[2];
  make_key(seed, key);
  return walk_normal(key, layout, node, path, j);
}

/* ------------------------------------------------------------------------ */
/* Coefficient functions: sum of products of elementary factors plus a dense
 * polynomial.  term_value() is one product without its coefficient. */
static double ipow(double v, int p) {
  double r = 1.0;
  for (int k = 0; k < p; ++k) r = r * v;
  return r;
}

static double factor_value(const orc_factor* fa, const double* x) {
  double s = fa->a * x[fa->dim] + fa->b;
  double v;
  switch (fa->fn) {
    case ORC_EXP: v = exp(s); break;
    case ORC_SIN: v = sin(s); break;
    case ORC_COS: v = cos(s); break;
    case ORC_TANH: v = tanh(s); break;
    default: v = s; break;
  }
  return ipow(v, fa->power);
}

static double term_value(const orc_fun* F, int t, const double* x) {
  double v = 1.0;
  for (int j = 0; j < F->n_factors; ++j) v = v * factor_value(&F->factors[t * F->n_factors + j], x);
  return v;
}

static double mono_value(const orc_fun* F, int m, const double* x) {
  const int32_t* e = &F->mono_exp[3 * m];
  return ipow(x[0], e[0]) * ipow(x[1], e[1]) * ipow(x[2], e[2]);
}

double orc_fun_eval(const orc_fun* F, const double* x) {
  double s = 0.0;
  for (int t = 0; t < F->n_terms; ++t) s += F->coef[t] * term_value(F, t, x);
  for (int m = 0; m < F->n_mono; ++m) s += F->mono_coef[m] * mono_value(F, m, x);
  return s;
}

/* ------------------------------------------------------------------------ */
/* Domain: D is open.  Box: lo_k < x_k < hi_k for all k.  Ball: |x - c|^2 < R^2.
 * A point on the boundary counts as outside (exited). */
int orc_inside(const orc_domain* D, const double* x) {
  if (D->kind == ORC_FREE) return 1;
  if (D->kind == ORC_BOX) {
    for (int k = 0; k < D->dim; ++k)
      if (!(x[k] > D->lo[k] && x[k] < D->hi[k])) return 0;
    return 1;
  }
  double r2 = 0.0;
  for (int k = 0; k < D->dim; ++k) {
    double d = x[k] - D->center[k];
    r2 += d * d;
  }
  return r2 < D->radius * D->radius;
}

/* Nearest point of the boundary.  Outside a box: clamp every coordinate.
 * Inside a box (only for a censored path): move the coordinate closest to a
 * face onto that face.  Ball: c + R (x - c)/|x - c| (c + R e_0 at the centre). */
void orc_project(const orc_domain* D, const double* x, double* out) {
  for (int k = 0; k < 3; ++k) out[k] = x[k];
  if (D->kind == ORC_BOX) {
    if (!orc_inside(D, x)) {
      for (int k = 0; k < D->dim; ++k) {
        if (out[k] < D->lo[k]) out[k] = D->lo[k];
        if (out[k] > D->hi[k]) out[k] = D->hi[k];
      }
    } else {
      int best = 0;
      double bestd = INFINITY, target = 0.0;
      for (int k = 0; k < D->dim; ++k) {
        double dl = x[k] - D->lo[k], dh = D->hi[k] - x[k];
        if (dl < bestd) { bestd = dl; best = k; target = D->lo[k]; }
        if (dh < bestd) { bestd = dh; best = k; target = D->hi[k]; }
      }
      out[best] = target;
    }
  } else if (D->kind == ORC_BALL) {
    double r2 = 0.0;
    for (int k = 0; k < D->dim; ++k) {
      double d = x[k] - D->center[k];
      r2 += d * d;
    }
    double r = sqrt(r2);
    if (r == 0.0) {
      out[0] = D->center[0] + D->radius;
      for (int k = 1; k < D->dim; ++k) out[k] = D->center[k];
    } else {
      for (int k = 0; k < D->dim; ++k) out[k] = D->center[k] + D->radius * (x[k] - D->center[k]) / r;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Tangents carried along one path for the adjoint (exact derivative of the
 * discrete estimator).  With Y_n = prod_{m<n} exp(-c(X_m) dt) and
 * Z_n = sum_{m<n} f(X_m) Y_m dt, and phi = g(X_tau) Y_N + Z_N:
 *   d phi / d coef_g[k]  = G_k(X_tau) Y_N
 *   d phi / d coef_f[j]  = F_j = sum_n m^f_j(X_n) Y_n dt
 *   d phi / d coef_c[j]  = -g(X_tau) Y_N S_j - A_j,
 *       S_j = sum_{n<N} m^c_j(X_n) dt,  A_j = sum_n f(X_n) Y_n dt S_j(n)
 * where S_j(n) is the partial sum before step n. */
typedef struct {
  int nf, nc;      /* parameter counts of f and c (terms then monomials) */
  double* F;
  double* S;
  double* A;
} tangents;

static double param_basis(const orc_fun* Fn, int j, const double* x) {
  if (j < Fn->n_terms) return term_value(Fn, j, x);
  return mono_value(Fn, j - Fn->n_terms, x);
}

typedef struct {
  double phi;
  int64_t steps;
  int censored;
  double xexit[3];
  double Y;
} path_result;

/* One path of the Feynman-Kac functional (Sec. 2.2, eqs. 2.7-2.9, elliptic
 * pure-Dirichlet limit, with c read as a killing rate: dY = -c Y dt):
 *   X_0 = node, Y_0 = 1, Z_0 = 0; for n = 0, 1, ...
 *     Z += f(X) Y dt;  Y *= exp(-c(X) dt);  X += b(X) dt + sigma sqrt(dt) zeta_n
 *   stopping at the first n with X outside D (or outside the shrunk test
 *   domain of the corrected scheme); then phi = g(P(X)) Y + Z with P the
 *   nearest-boundary projection onto dD.  A node outside D gives phi = g(P(node)).
 *   A path reaching max_steps is censored: phi = g(P(X)) Y + Z. */
/* The domain of the exit test: D itself, or D shrunk by c0 sigma sqrt(dt)
 * for the boundary-corrected scheme (Sec. 2.1 points to Gobet and Menozzi's
 * corrected Euler schemes for stopped diffusions; their correction moves the
 * boundary inward by c0 |sigma n| sqrt(dt), c0 = -zeta(1/2)/sqrt(2 pi), and
 * |sigma n| = sigma here since the diffusion matrix is sigma I). */
static orc_domain test_domain(const orc_linear* P, double dt) {
  orc_domain T = P->dom;
  if (P->boundary_shift > 0.0) {
    const double delta = P->boundary_shift * P->sigma * sqrt(dt);
    if (T.kind == ORC_BOX) {
      for (int k = 0; k < T.dim; ++k) {
        T.lo[k] = T.lo[k] + delta;
        T.hi[k] = T.hi[k] - delta;
      }
    } else if (T.kind == ORC_BALL) {
      T.radius = T.radius - delta;
      if (T.radius < 0.0) T.radius = 0.0;
    }
  }
  return T;
}

static path_result walk_path(const orc_linear* P, const double* node, const uint32_t key[2], int layout,
                             uint32_t node_idx, uint32_t path_idx, double dt, int64_t max_steps,
                             tangents* tg) {
  path_result R;
  const orc_domain* D = &P->dom;
  const orc_domain DT = test_domain(P, dt);
  int d = D->dim;
  double X[3] = {0.0, 0.0, 0.0}, Xp[3];
  for (int k = 0; k < d; ++k) X[k] = node[k];
  double Y = 1.0, Z = 0.0;
  int64_t n = 0;
  double sdt = sqrt(dt);
  R.censored = 0;
  if (tg) {
    for (int j = 0; j < tg->nf; ++j) tg->F[j] = 0.0;
    for (int j = 0; j < tg->nc; ++j) { tg->S[j] = 0.0; tg->A[j] = 0.0; }
  }
  if (!orc_inside(&DT, X)) {
    orc_project(D, X, Xp);
    R.phi = orc_fun_eval(&P->g, Xp);
    R.steps = 0;
    for (int k = 0; k < 3; ++k) R.xexit[k] = Xp[k];
    R.Y = 1.0;
    return R;
  }
  for (;;) {
    if (n == max_steps) { R.censored = 1; break; }
    double zeta[3];
    for (int k = 0; k < d; ++k) zeta[k] = walk_normal(key, layout, node_idx, path_idx, (uint64_t)n * d + k);
    double fx = orc_fun_eval(&P->f, X);
    double cx = orc_fun_eval(&P->c, X);
    if (tg) {
      for (int j = 0; j < tg->nc; ++j) tg->A[j] += fx * Y * dt * tg->S[j];
      for (int j = 0; j < tg->nf; ++j) tg->F[j] += param_basis(&P->f, j, X) * Y * dt;
      for (int j = 0; j < tg->nc; ++j) tg->S[j] += param_basis(&P->c, j, X) * dt;
    }
    Z = Z + fx * Y * dt;
    Y = Y * exp(-cx * dt);
    double bx[3];
    for (int k = 0; k < d; ++k) bx[k] = orc_fun_eval(&P->b[k], X);
    for (int k = 0; k < d; ++k) X[k] = X[k] + bx[k] * dt + P->sigma * sdt * zeta[k];
    n += 1;
    if (!orc_inside(&DT, X)) break;
  }
  orc_project(D, X, Xp);
  R.phi = orc_fun_eval(&P->g, Xp) * Y + Z;
  R.steps = n;
  for (int k = 0; k < 3; ++k) R.xexit[k] = Xp[k];
  R.Y = Y;
  return R;
}

/* Welford's running mean / sum of squared deviations, in path order. */
static void welford_push(orc_stat* s, double x) {
  s->n += 1;
  double delta = x - s->mean;
  s->mean += delta / (double)s->n;
  s->m2 += delta * (x - s->mean);
}

/* ------------------------------------------------------------------------ */
/* Tiny thread pool: workers pull item indices from a shared counter.  Each
 * item's result depends only on the item, never on the worker. */
typedef struct {
  void (*fn)(void* ctx, int64_t item, int worker);
  void* ctx;
  int64_t n_items;
  int64_t next;
  pthread_mutex_t mu;
  int worker;
} pool_job;

typedef struct { pool_job* job; int id; } pool_arg;

static void* pool_worker(void* p) {
  pool_arg* a = (pool_arg*)p;
  pool_job* job = a->job;
  for (;;) {
    pthread_mutex_lock(&job->mu);
    int64_t i = job->next++;
    pthread_mutex_unlock(&job->mu);
    if (i >= job->n_items) break;
    job->fn(job->ctx, i, a->id);
  }
  return NULL;
}

static void run_pool(int n_threads, int64_t n_items, void (*fn)(void*, int64_t, int), void* ctx) {
  if (n_threads < 1) n_threads = 1;
  if (n_threads == 1 || n_items <= 1) {
    for (int64_t i = 0; i < n_items; ++i) fn(ctx, i, 0);
    return;
  }
  pool_job job;
  job.fn = fn; job.ctx = ctx; job.n_items = n_items; job.next = 0;
  pthread_mutex_init(&job.mu, NULL);
  pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)n_threads);
  pool_arg* args = (pool_arg*)malloc(sizeof(pool_arg) * (size_t)n_threads);
  for (int t = 0; t < n_threads; ++t) {
    args[t].job = &job; args[t].id = t;
    pthread_create(&th[t], NULL, pool_worker, &args[t]);
  }
  for (int t = 0; t < n_threads; ++t) pthread_join(th[t], NULL);
  pthread_mutex_destroy(&job.mu);
  free(th); free(args);
}

/* ------------------------------------------------------------------------ */
typedef struct {
  const orc_linear* P;
  const double* nodes;
  const int64_t* paths;
  const int64_t* offsets;
  double dt;
  uint32_t key[2];
  int layout;
  int64_t max_steps;
  orc_stat* out;
  double* dump_phi;
  int64_t* dump_steps;
  /* adjoint */
  const double* w;
  double* grad_rows;   /* [n_nodes][n_grad] */
  int n_grad;
  const int64_t* node_ids; /* counter word 3 per node (NULL: the node's position) */
  void* extra;             /* per-function outputs (orc_walk_jacobian) */
} walk_ctx;

static uint32_t node_id(const walk_ctx* C, int64_t i) { return (uint32_t)(C->node_ids ? C->node_ids[i] : i); }

static void walk_node(void* vctx, int64_t i, int worker) {
  (void)worker;
  walk_ctx* C = (walk_ctx*)vctx;
  int d = C->P->dom.dim;
  orc_stat s = {0.0, 0.0, 0, 0, 0};
  for (int64_t p = 0; p < C->paths[i]; ++p) {
    path_result R = walk_path(C->P, &C->nodes[i * d], C->key, C->layout, node_id(C, i), (uint32_t)p,
                              C->dt, C->max_steps, NULL);
    welford_push(&s, R.phi);
    s.steps += R.steps;
    s.censored += R.censored;
    if (C->dump_phi) C->dump_phi[C->offsets[i] + p] = R.phi;
    if (C->dump_steps) C->dump_steps[C->offsets[i] + p] = R.steps;
  }
  C->out[i] = s;
}

static int64_t* prefix_offsets(const int64_t* paths, int64_t n) {
  int64_t* off = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
  off[0] = 0;
  for (int64_t i = 0; i < n; ++i) off[i + 1] = off[i] + paths[i];
  return off;
}

int orc_walk(const orc_linear* P, const double* nodes, int64_t n_nodes, const int64_t* paths,
             double dt, uint64_t seed, int layout, int64_t max_steps, int n_threads,
             orc_stat* out, double* dump_phi, int64_t* dump_steps, const int64_t* node_ids) {
  if (P->dom.kind == ORC_FREE || P->dom.dim < 1 || P->dom.dim > 3 || !(dt > 0.0)) return -1;
  walk_ctx C;
  memset(&C, 0, sizeof(C));
  C.P = P; C.nodes = nodes; C.paths = paths; C.dt = dt; C.layout = layout;
  C.max_steps = max_steps; C.out = out; C.dump_phi = dump_phi; C.dump_steps = dump_steps;
  C.node_ids = node_ids;
  make_key(seed, C.key);
  int64_t* off = prefix_offsets(paths, n_nodes);
  C.offsets = off;
  run_pool(n_threads, n_nodes, walk_node, &C);
  free(off);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Walk on Spheres.  Distance to the boundary of the open set D: ball
 * R - |x - c|, box min_k min(x_k - lo_k, hi_k - x_k) (negative outside). */
static double boundary_distance(const orc_domain* D, const double* x) {
  if (D->kind == ORC_BALL) {
    double r2 = 0.0;
    for (int k = 0; k < D->dim; ++k) {
      double v = x[k] - D->center[k];
      r2 += v * v;
    }
    return D->radius - sqrt(r2);
  }
  double m = INFINITY;
  for (int k = 0; k < D->dim; ++k) {
    double lo = x[k] - D->lo[k], hi = D->hi[k] - x[k];
    if (lo < m) m = lo;
    if (hi < m) m = hi;
  }
  return m;
}

static int fun_is_zero(const orc_fun* F) { return F->n_terms == 0 && F->n_mono == 0; }

static void wos_node(void* vctx, int64_t i, int worker) {
  (void)worker;
  walk_ctx* C = (walk_ctx*)vctx;
  const orc_linear* P = C->P;
  const orc_domain* D = &P->dom;
  int d = D->dim;
  double eps = C->dt;
  orc_stat s = {0.0, 0.0, 0, 0, 0};
  for (int64_t p = 0; p < C->paths[i]; ++p) {
    double X[3] = {0.0, 0.0, 0.0}, Xp[3];
    for (int k = 0; k < d; ++k) X[k] = C->nodes[i * d + k];
    int64_t n = 0;
    int censored = 0;
    if (orc_inside(D, X)) {
      for (;;) {
        double r = boundary_distance(D, X);
        if (r < eps) break;
        if (n == C->max_steps) { censored = 1; break; }
        double zeta[3], z2 = 0.0;
        for (int k = 0; k < d; ++k) {
          zeta[k] = walk_normal(C->key, C->layout, node_id(C, i), (uint32_t)p, (uint64_t)n * d + k);
          z2 += zeta[k] * zeta[k];
        }
        double zn = sqrt(z2);
        for (int k = 0; k < d; ++k) X[k] = X[k] + r * (zeta[k] / zn);
        n += 1;
      }
    }
    orc_project(D, X, Xp);
    double phi = orc_fun_eval(&P->g, Xp);
    welford_push(&s, phi);
    s.steps += n;
    s.censored += censored;
    if (C->dump_phi) C->dump_phi[C->offsets[i] + p] = phi;
    if (C->dump_steps) C->dump_steps[C->offsets[i] + p] = n;
  }
  C->out[i] = s;
}

int orc_wos(const orc_linear* P, const double* nodes, int64_t n_nodes, const int64_t* paths,
            double eps, uint64_t seed, int layout, int64_t max_steps, int n_threads,
            orc_stat* out, double* dump_phi, int64_t* dump_steps, const int64_t* node_ids) {
  if ((P->dom.kind != ORC_BOX && P->dom.kind != ORC_BALL) || P->dom.dim < 1 || P->dom.dim > 3 || !(eps > 0.0))
    return -1;
  for (int k = 0; k < P->dom.dim; ++k)
    if (!fun_is_zero(&P->b[k])) return -1;
  if (!fun_is_zero(&P->c) || !fun_is_zero(&P->f)) return -1;
  walk_ctx C;
  memset(&C, 0, sizeof(C));
  C.P = P; C.nodes = nodes; C.paths = paths; C.dt = eps; C.layout = layout;
  C.max_steps = max_steps; C.out = out; C.dump_phi = dump_phi; C.dump_steps = dump_steps;
  C.node_ids = node_ids;
  make_key(seed, C.key);
  int64_t* off = prefix_offsets(paths, n_nodes);
  C.offsets = off;
  run_pool(n_threads, n_nodes, wos_node, &C);
  free(off);
  return 0;
}

/* ------------------------------------------------------------------------ */
static int fun_params(const orc_fun* F) { return F->n_terms + F->n_mono; }

static void adjoint_node(void* vctx, int64_t i, int worker) {
  (void)worker;
  walk_ctx* C = (walk_ctx*)vctx;
  const orc_linear* P = C->P;
  int d = P->dom.dim;
  int ng = fun_params(&P->g), nf = fun_params(&P->f), nc = fun_params(&P->c);
  double* row = &C->grad_rows[i * C->n_grad];
  double* Fj = (double*)calloc((size_t)(nf + 2 * nc + ng + 1), sizeof(double));
  tangents tg;
  tg.nf = nf; tg.nc = nc; tg.F = Fj; tg.S = Fj + nf; tg.A = Fj + nf + nc;
  double* gk = Fj + nf + 2 * nc;
  orc_stat s = {0.0, 0.0, 0, 0, 0};
  double wN = C->w[i] / (double)C->paths[i];
  for (int64_t p = 0; p < C->paths[i]; ++p) {
    path_result R = walk_path(P, &C->nodes[i * d], C->key, C->layout, node_id(C, i), (uint32_t)p,
                              C->dt, C->max_steps, &tg);
    welford_push(&s, R.phi);
    s.steps += R.steps;
    s.censored += R.censored;
    double gval = orc_fun_eval(&P->g, R.xexit);
    for (int k = 0; k < ng; ++k) gk[k] = param_basis(&P->g, k, R.xexit);
    /* row layout: [g params | f params | c params] */
    for (int k = 0; k < ng; ++k) row[k] += wN * gk[k] * R.Y;
    for (int j = 0; j < nf; ++j) row[ng + j] += wN * tg.F[j];
    for (int j = 0; j < nc; ++j) row[ng + nf + j] += wN * (-gval * R.Y * tg.S[j] - tg.A[j]);
  }
  if (C->out) C->out[i] = s;
  free(Fj);
}

int orc_walk_adjoint(const orc_linear* P, const double* nodes, int64_t n_nodes, const int64_t* paths,
                     double dt, uint64_t seed, int layout, int64_t max_steps, int n_threads,
                     const double* w,
                     double* dg_coef, double* dg_mono, double* df_coef, double* df_mono,
                     double* dc_coef, double* dc_mono, orc_stat* out) {
  if (P->dom.kind == ORC_FREE || P->dom.dim < 1 || P->dom.dim > 3 || !(dt > 0.0)) return -1;
  walk_ctx C;
  memset(&C, 0, sizeof(C));
  C.P = P; C.nodes = nodes; C.paths = paths; C.dt = dt; C.layout = layout;
  C.max_steps = max_steps; C.out = out; C.w = w;
  make_key(seed, C.key);
  int ng = fun_params(&P->g), nf = fun_params(&P->f), nc = fun_params(&P->c);
  C.n_grad = ng + nf + nc;
  C.grad_rows = (double*)calloc((size_t)(n_nodes * C.n_grad + 1), sizeof(double));
  run_pool(n_threads, n_nodes, adjoint_node, &C);
  /* sum the per-node rows in node order */
  for (int64_t i = 0; i < n_nodes; ++i) {
    const double* row = &C.grad_rows[i * C.n_grad];
    for (int k = 0; k < P->g.n_terms; ++k) if (dg_coef) dg_coef[k] += row[k];
    for (int k = 0; k < P->g.n_mono; ++k) if (dg_mono) dg_mono[k] += row[P->g.n_terms + k];
    for (int k = 0; k < P->f.n_terms; ++k) if (df_coef) df_coef[k] += row[ng + k];
    for (int k = 0; k < P->f.n_mono; ++k) if (df_mono) df_mono[k] += row[ng + P->f.n_terms + k];
    for (int k = 0; k < P->c.n_terms; ++k) if (dc_coef) dc_coef[k] += row[ng + nf + k];
    for (int k = 0; k < P->c.n_mono; ++k) if (dc_mono) dc_mono[k] += row[ng + nf + P->c.n_terms + k];
  }
  free(C.grad_rows);
  return 0;
}

/* Per-node Jacobian with the spread of the per-path derivatives.  The
 * derivative of one path value is the one the adjoint sums (exact derivative
 * of the discrete estimator): G_k(X_tau) Y_N for a coefficient of g, F_j for
 * one of f, -g(X_tau) Y_N S_j - A_j for one of c.  Each is pushed into its
 * own Welford accumulator, in path order. */
typedef struct {
  double* mean;   /* [n_nodes][n_grad] */
  double* m2;
} jac_out;

static void jacobian_node(void* vctx, int64_t i, int worker) {
  (void)worker;
  walk_ctx* C = (walk_ctx*)vctx;
  const jac_out* J = (const jac_out*)C->extra;
  const orc_linear* P = C->P;
  int d = P->dom.dim;
  int ng = fun_params(&P->g), nf = fun_params(&P->f), nc = fun_params(&P->c);
  int np = ng + nf + nc;
  double* mean = &J->mean[i * np];
  double* m2 = &J->m2[i * np];
  double* Fj = (double*)calloc((size_t)(nf + 2 * nc + np + 1), sizeof(double));
  tangents tg;
  tg.nf = nf; tg.nc = nc; tg.F = Fj; tg.S = Fj + nf; tg.A = Fj + nf + nc;
  double* dphi = Fj + nf + 2 * nc;
  orc_stat s = {0.0, 0.0, 0, 0, 0};
  for (int k = 0; k < np; ++k) { mean[k] = 0.0; m2[k] = 0.0; }
  for (int64_t p = 0; p < C->paths[i]; ++p) {
    path_result R = walk_path(P, &C->nodes[i * d], C->key, C->layout, node_id(C, i), (uint32_t)p,
                              C->dt, C->max_steps, &tg);
    welford_push(&s, R.phi);
    s.steps += R.steps;
    s.censored += R.censored;
    double gval = orc_fun_eval(&P->g, R.xexit);
    for (int k = 0; k < ng; ++k) dphi[k] = param_basis(&P->g, k, R.xexit) * R.Y;
    for (int j = 0; j < nf; ++j) dphi[ng + j] = tg.F[j];
    for (int j = 0; j < nc; ++j) dphi[ng + nf + j] = -gval * R.Y * tg.S[j] - tg.A[j];
    double cnt = (double)(p + 1);
    for (int k = 0; k < np; ++k) {
      double delta = dphi[k] - mean[k];
      mean[k] += delta / cnt;
      m2[k] += delta * (dphi[k] - mean[k]);
    }
  }
  if (C->out) C->out[i] = s;
  free(Fj);
}

int orc_walk_jacobian(const orc_linear* P, const double* nodes, int64_t n_nodes, const int64_t* paths,
                      double dt, uint64_t seed, int layout, int64_t max_steps, int n_threads,
                      double* jac_mean, double* jac_m2, orc_stat* out, const int64_t* node_ids) {
  if (P->dom.kind == ORC_FREE || P->dom.dim < 1 || P->dom.dim > 3 || !(dt > 0.0)) return -1;
  walk_ctx C;
  memset(&C, 0, sizeof(C));
  C.P = P; C.nodes = nodes; C.paths = paths; C.dt = dt; C.layout = layout;
  C.max_steps = max_steps; C.out = out; C.node_ids = node_ids;
  make_key(seed, C.key);
  jac_out J = {jac_mean, jac_m2};
  C.extra = &J;
  run_pool(n_threads, n_nodes, jacobian_node, &C);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Branching diffusion, per-particle (depth-first) form.
 *
 * Sec. 3.1 describes the particle system: a particle started at x lives an
 * Exp(beta) time, moves as a diffusion with generator 0.5 sigma^2 Lap (exact
 * Brownian increments, since the driving process is Brownian motion), and at
 * its death branches into i particles with probability alpha_i.  Eq. 3.1's
 * solution at time T is E[prod over particles alive at T of psi(X_T)].  The
 * marked form of Sec. 3.2 samples the offspring count from q instead and
 * multiplies the weight by alpha_I / q_I at each branching.
 *
 * Randomness is addressed by the particle's label l (root 1, the i-th child of
 * l is B*l + i with B = max(2, largest offspring count)), so the tree does not
 * depend on the order in which particles are simulated.  Counter words:
 * word0 = low 32 bits of l, word1 = stream << 24 | attempt << 20 | blk << 16 |
 * bits 32..47 of l, word2 = tree index, word3 = point index.  Stream 1 gives
 * the lifetime and type uniforms, stream 2 the Gaussians.
 *
 * Pruning (the remark before Algorithm 3.1, and the restart step inside it):
 * a tree that needs more than max_segments particles, or a label of 48 bits or
 * more, is discarded and drawn again with attempt + 1; after 15 redraws the
 * tree counts as censored with value 0. */
#define BR_MAX_STACK 4096

typedef struct { uint64_t label; double x[3]; double t; } br_seg;

static void branch_uniforms(const uint32_t key[2], int layout, uint64_t label, int attempt, uint32_t tree,
                            uint32_t point, double* ulife, double* utype) {
  uint32_t ctr[4], w[4];
  ctr[0] = (uint32_t)label;
  ctr[1] = (1u << 24) | ((uint32_t)attempt << 20) | (0u << 16) | (uint32_t)((label >> 32) & 0xFFFFu);
  ctr[2] = tree; ctr[3] = point;
  orc_philox4x32_10(ctr, key, w);
  if (layout == ORC_QUAD24) {
    *ulife = u_quad24(w[0]);
    *utype = u_quad24(w[1]);
  } else {
    *ulife = u_pair52(w[0], w[1]);
    *utype = u_pair52(w[2], w[3]);
  }
}

static void branch_normals(const uint32_t key[2], int layout, uint64_t label, int attempt, uint32_t tree,
                           uint32_t point, int d, double* z) {
  uint32_t ctr[4], w[4];
  double tmp[4];
  ctr[0] = (uint32_t)label;
  ctr[2] = tree; ctr[3] = point;
  if (layout == ORC_QUAD24) {
    ctr[1] = (2u << 24) | ((uint32_t)attempt << 20) | (0u << 16) | (uint32_t)((label >> 32) & 0xFFFFu);
    orc_philox4x32_10(ctr, key, w);
    box_muller(u_quad24(w[0]), u_quad24(w[1]), &tmp[0], &tmp[1]);
    box_muller(u_quad24(w[2]), u_quad24(w[3]), &tmp[2], &tmp[3]);
  } else {
    for (uint32_t blk = 0; blk < 2; ++blk) {
      ctr[1] = (2u << 24) | ((uint32_t)attempt << 20) | (blk << 16) | (uint32_t)((label >> 32) & 0xFFFFu);
      orc_philox4x32_10(ctr, key, w);
      box_muller(u_pair52(w[0], w[1]), u_pair52(w[2], w[3]), &tmp[2 * blk], &tmp[2 * blk + 1]);
    }
  }
  for (int k = 0; k < d; ++k) z[k] = tmp[k];
}

/* offspring count: the smallest k with u < q_0 + ... + q_k (the last k with
 * q_k > 0 if rounding leaves u above the total). */
static int pick_type(const double* q, double u) {
  double cum = 0.0;
  int last = 0;
  for (int k = 0; k < 5; ++k) {
    if (q[k] > 0.0) last = k;
    cum += q[k];
    if (q[k] > 0.0 && u < cum) return k;
  }
  return last;
}

static int label_base(const orc_branching* B) {
  int L = 0;
  for (int k = 0; k < 5; ++k) if (B->q[k] > 0.0) L = k;
  return L < 2 ? 2 : L;
}

typedef struct {
  const orc_branching* B;
  const double* points;
  int64_t trees;
  uint32_t key[2];
  int layout;
  int max_particles;
  orc_stat* out;
  double* dump_val;
  int64_t* dump_segs;
  int64_t* redrawn_per_point;
} br_ctx;

/* one tree; returns 0 on success, 1 if the cap was hit */
static int tree_once(const orc_branching* B, const double* x0, const uint32_t key[2], int layout, int attempt,
                     uint32_t tree, uint32_t point, br_seg* stack, double* value, int64_t* segs_out) {
  int d = B->dim;
  uint64_t base = (uint64_t)label_base(B);
  int top = 0;
  stack[0].label = 1;
  for (int k = 0; k < 3; ++k) stack[0].x[k] = (k < d) ? x0[k] : 0.0;
  stack[0].t = 0.0;
  top = 1;
  double W = 1.0, prod = 1.0;
  int64_t segs = 0;
  double sq = B->sigma;
  while (top > 0) {
    br_seg s = stack[--top];
    segs += 1;
    if (segs > B->max_segments) { *segs_out = segs; return 1; }
    double ulife, utype, z[3];
    branch_uniforms(key, layout, s.label, attempt, tree, point, &ulife, &utype);
    branch_normals(key, layout, s.label, attempt, tree, point, d, z);
    double E = -log(ulife) / B->beta;
    double rem = B->T - s.t;
    double delta = (E < rem) ? E : rem;
    double sd = sq * sqrt(delta);
    for (int k = 0; k < d; ++k) s.x[k] = s.x[k] + sd * z[k];
    if (E < rem) {
      int I = pick_type(B->q, utype);
      W = W * (B->alpha[I] / B->q[I]);
      for (int i = I - 1; i >= 0; --i) {
        uint64_t child = base * s.label + (uint64_t)i;
        if (child >= (1ull << 48) || s.label >= (1ull << 47) || top >= BR_MAX_STACK) { *segs_out = segs; return 1; }
        stack[top].label = child;
        for (int k = 0; k < 3; ++k) stack[top].x[k] = s.x[k];
        stack[top].t = s.t + E;
        top++;
      }
    } else {
      prod = prod * orc_fun_eval(&B->psi, s.x);
    }
  }
  *value = prod * W;
  *segs_out = segs;
  return 0;
}

static void branching_point(void* vctx, int64_t i, int worker) {
  (void)worker;
  br_ctx* C = (br_ctx*)vctx;
  const orc_branching* B = C->B;
  br_seg* stack = (br_seg*)malloc(sizeof(br_seg) * BR_MAX_STACK);
  orc_stat s = {0.0, 0.0, 0, 0, 0};
  int64_t redrawn = 0;
  for (int64_t t = 0; t < C->trees; ++t) {
    double value = 0.0;
    int64_t segs = 0;
    int attempt = 0, ok = 0;
    for (attempt = 0; attempt < 16; ++attempt) {
      if (tree_once(B, &C->points[i * B->dim], C->key, C->layout, attempt, (uint32_t)t, (uint32_t)i, stack,
                    &value, &segs) == 0) { ok = 1; break; }
      redrawn += 1;
    }
    if (!ok) { value = 0.0; s.censored += 1; }
    welford_push(&s, value);
    s.steps += segs;
    if (C->dump_val) C->dump_val[i * C->trees + t] = value;
    if (C->dump_segs) C->dump_segs[i * C->trees + t] = segs;
  }
  C->out[i] = s;
  C->redrawn_per_point[i] = redrawn;
  free(stack);
}

int orc_branching_dfs(const orc_branching* B, const double* points, int64_t n_points,
                      int64_t trees, uint64_t seed, int layout, int n_threads,
                      orc_stat* out, double* dump_val, int64_t* dump_segs, int64_t* redrawn) {
  if (B->dim < 1 || B->dim > 3 || !(B->beta > 0.0) || !(B->T >= 0.0)) return -1;
  br_ctx C;
  memset(&C, 0, sizeof(C));
  C.B = B; C.points = points; C.trees = trees; C.layout = layout; C.out = out;
  C.dump_val = dump_val; C.dump_segs = dump_segs;
  C.redrawn_per_point = (int64_t*)calloc((size_t)n_points + 1, sizeof(int64_t));
  make_key(seed, C.key);
  run_pool(n_threads, n_points, branching_point, &C);
  int64_t tot = 0;
  for (int64_t i = 0; i < n_points; ++i) tot += C.redrawn_per_point[i];
  if (redrawn) *redrawn = tot;
  free(C.redrawn_per_point);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Global-clock form (Algorithm 3.1): with N_p particles alive at time t, the
 * next branching happens after an Exp(beta N_p) time; if that is before T,
 * every particle moves by an exact Brownian increment over the waiting time, a
 * particle chosen uniformly branches (offspring count from q, weight times
 * alpha_I / q_I); otherwise all particles move to T and the sample is the
 * weight times the product of psi over them.  More than max_particles alive
 * restarts the sample (attempt + 1).  Its own counter use:
 * word0 = event index, word1 = stream << 24 | attempt << 20 | blk << 16 |
 * particle, with stream 3 for clock/choice/type uniforms and stream 4 for the
 * Gaussians (particle < 2^16). */
static void alg31_uniforms(const uint32_t key[2], uint32_t ev, int attempt, uint32_t tree, uint32_t point,
                           double* u) {
  uint32_t ctr[4], w[4];
  ctr[0] = ev;
  ctr[1] = (3u << 24) | ((uint32_t)attempt << 20);
  ctr[2] = tree; ctr[3] = point;
  orc_philox4x32_10(ctr, key, w);
  u[0] = u_pair52(w[0], w[1]);
  u[1] = u_quad24(w[2]);
  u[2] = u_quad24(w[3]);
}

static void alg31_normals(const uint32_t key[2], uint32_t ev, int attempt, uint32_t particle, uint32_t tree,
                          uint32_t point, int d, double* z) {
  uint32_t ctr[4], w[4];
  double tmp[4];
  ctr[0] = ev;
  ctr[2] = tree; ctr[3] = point;
  for (uint32_t blk = 0; blk < 2; ++blk) {
    ctr[1] = (4u << 24) | ((uint32_t)attempt << 20) | (blk << 16) | (particle & 0xFFFFu);
    orc_philox4x32_10(ctr, key, w);
    box_muller(u_pair52(w[0], w[1]), u_pair52(w[2], w[3]), &tmp[2 * blk], &tmp[2 * blk + 1]);
  }
  for (int k = 0; k < d; ++k) z[k] = tmp[k];
}

static int alg31_once(const orc_branching* B, const double* x0, const uint32_t key[2], int attempt,
                      uint32_t tree, uint32_t point, int maxp, double* pos, double* value, int64_t* events) {
  int d = B->dim;
  int np = 1;
  for (int k = 0; k < d; ++k) pos[k] = x0[k];
  double t = 0.0, W = 1.0;
  uint32_t ev = 0;
  for (;;) {
    double u[3], z[3];
    alg31_uniforms(key, ev, attempt, tree, point, u);
    double tc = (np > 0) ? -log(u[0]) / (B->beta * (double)np) : INFINITY;
    double step = (t + tc < B->T) ? tc : (B->T - t);
    double sd = B->sigma * sqrt(step);
    for (int j = 0; j < np; ++j) {
      alg31_normals(key, ev, attempt, (uint32_t)j, tree, point, d, z);
      for (int k = 0; k < d; ++k) pos[j * 3 + k] = pos[j * 3 + k] + sd * z[k];
    }
    if (!(t + tc < B->T)) {
      double prod = 1.0;
      for (int j = 0; j < np; ++j) prod = prod * orc_fun_eval(&B->psi, &pos[j * 3]);
      *value = prod * W;
      *events = ev;
      return 0;
    }
    t = t + tc;
    int pick = (int)(u[1] * (double)np);
    if (pick >= np) pick = np - 1;
    int I = pick_type(B->q, u[2]);
    W = W * (B->alpha[I] / B->q[I]);
    if (np - 1 + I > maxp) { *events = ev; return 1; }
    double px[3] = {pos[pick * 3], pos[pick * 3 + 1], pos[pick * 3 + 2]};
    /* remove the picked particle (move the last one into its slot), then append I copies */
    for (int k = 0; k < 3; ++k) pos[pick * 3 + k] = pos[(np - 1) * 3 + k];
    np -= 1;
    for (int i = 0; i < I; ++i) {
      for (int k = 0; k < 3; ++k) pos[np * 3 + k] = px[k];
      np += 1;
    }
    ev += 1;
  }
}

static void alg31_point(void* vctx, int64_t i, int worker) {
  (void)worker;
  br_ctx* C = (br_ctx*)vctx;
  const orc_branching* B = C->B;
  double* pos = (double*)malloc(sizeof(double) * 3 * (size_t)(C->max_particles + 8));
  orc_stat s = {0.0, 0.0, 0, 0, 0};
  int64_t redrawn = 0;
  for (int64_t t = 0; t < C->trees; ++t) {
    double value = 0.0;
    int64_t ev = 0;
    int ok = 0;
    for (int attempt = 0; attempt < 16; ++attempt) {
      if (alg31_once(B, &C->points[i * B->dim], C->key, attempt, (uint32_t)t, (uint32_t)i, C->max_particles,
                     pos, &value, &ev) == 0) { ok = 1; break; }
      redrawn += 1;
    }
    if (!ok) { value = 0.0; s.censored += 1; }
    welford_push(&s, value);
    s.steps += ev;
  }
  C->out[i] = s;
  C->redrawn_per_point[i] = redrawn;
  free(pos);
}

int orc_branching_alg31(const orc_branching* B, const double* points, int64_t n_points,
                        int64_t trees, uint64_t seed, int max_particles, int n_threads,
                        orc_stat* out, int64_t* redrawn) {
  if (B->dim < 1 || B->dim > 3 || !(B->beta > 0.0) || max_particles < 1 || max_particles > 60000) return -1;
  br_ctx C;
  memset(&C, 0, sizeof(C));
  C.B = B; C.points = points; C.trees = trees; C.max_particles = max_particles; C.out = out;
  C.redrawn_per_point = (int64_t*)calloc((size_t)n_points + 1, sizeof(int64_t));
  make_key(seed, C.key);
  run_pool(n_threads, n_points, alg31_point, &C);
  int64_t tot = 0;
  for (int64_t i = 0; i < n_points; ++i) tot += C.redrawn_per_point[i];
  if (redrawn) *redrawn = tot;
  free(C.redrawn_per_point);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Branching with a Dirichlet boundary and several output times (eq. 3.2 and
 * Algorithm 3.1).  Eq. 3.2: the particles of the branching system started at
 * x are stopped when they reach the boundary of the domain; the estimator of
 * u(x, t) is the product, over the particles present at time t, of psi(X_t)
 * for those still inside and g(X_tau, t - tau) for those stopped at time tau
 * (times the marks alpha_I / q_I of every branching before t, Sec. 3.2).
 * Algorithm 3.1 evaluates one simulated tree at every output time t_i.
 *
 * Scheme (the paper gives the representation, not a discretisation): a
 * particle born at time s0 with lifetime E (stream 1, as in the free-space
 * estimator) moves by exact Brownian increments over sub-steps that end at
 * min(s + dt, its death time s0 + E, the horizon t_last, the next output time
 * t_k > s), and is tested against the boundary after every sub-step; a
 * particle found outside is projected onto the boundary and stopped at the
 * end time s of that sub-step (the linear walk's exit rule).  For every
 * output time t_i >= s its factor is g(P X, t_i - s).  A particle still inside
 * when a sub-step ends on t_k multiplies factor k by psi(X).  The sub-step
 * that ends at the particle's death (before t_last) is not tested: the
 * offspring count I is drawn from q, every output time after the death picks
 * up alpha_I / q_I, and the children start at X, where each is tested at its
 * birth (a particle born outside is stopped at its birth time s0 with factor
 * g(P X, t_i - s0)).  Testing at the death instead, before branching, would
 * look ahead to the death time and bias the estimator by O(dt) even for
 * spatially constant solutions.  The start point is tested the same way; an
 * output time t_i = 0 takes psi(x) when it is inside.  With boundary_shift =
 * c0 > 0 the test after a sub-step of length h uses the domain shrunk by
 * c0 sigma sqrt(h) (the walk's boundary correction, per sub-step); the test
 * at birth uses the domain itself.
 *
 * Gaussians of a particle: number n d + k (sub-step n, coordinate k) comes
 * from Philox block j = (n d + k) / m, slot (n d + k) mod m (m = 4 for the
 * QUAD24 lattice, 2 for PAIR52), counter word0 = low 32 bits of the label,
 * word1 = 5 << 28 | attempt << 24 | bits 32..47 of the label << 8 | bits 8..15
 * of j, word2 = tree, word3 = point (24 bits) | bits 0..7 of j << 24 (stream
 * 5; j < 2^16, point < 2^24).  Segment count, pruning and redraws as in the
 * free-space estimator; a censored tree is 0 at every output time. */
static double bvp_normal(const uint32_t key[2], int layout, uint64_t label, int attempt, uint32_t tree,
                         uint32_t point, uint64_t g) {
  const uint64_t per = (layout == ORC_QUAD24) ? 4 : 2;
  const uint32_t j = (uint32_t)(g / per);
  const int slot = (int)(g % per);
  uint32_t ctr[4], w[4];
  double tmp[4];
  ctr[0] = (uint32_t)label;
  ctr[1] = (5u << 28) | ((uint32_t)attempt << 24) | ((uint32_t)((label >> 32) & 0xFFFFu) << 8) | ((j >> 8) & 0xFFu);
  ctr[2] = tree;
  ctr[3] = (point & 0xFFFFFFu) | ((j & 0xFFu) << 24);
  orc_philox4x32_10(ctr, key, w);
  if (layout == ORC_QUAD24) {
    box_muller(u_quad24(w[0]), u_quad24(w[1]), &tmp[0], &tmp[1]);
    box_muller(u_quad24(w[2]), u_quad24(w[3]), &tmp[2], &tmp[3]);
  } else {
    box_muller(u_pair52(w[0], w[1]), u_pair52(w[2], w[3]), &tmp[0], &tmp[1]);
  }
  return tmp[slot];
}

/* inside the domain shrunk by delta (box: every face moved in; ball: radius
 * R - delta, at least 0) */
static int inside_shrunk(const orc_domain* D, const double* x, double delta) {
  orc_domain S = *D;
  for (int k = 0; k < 3; ++k) { S.lo[k] += delta; S.hi[k] -= delta; }
  S.radius = D->radius - delta > 0.0 ? D->radius - delta : 0.0;
  return orc_inside(&S, x);
}

/* g at (boundary point, time argument): the time is coordinate index dim */
static double bvp_g(const orc_branch_boundary* Bd, int d, const double* xp, double s) {
  double xs[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k = 0; k < d; ++k) xs[k] = xp[k];
  xs[d] = s;
  return orc_fun_eval(&Bd->g, xs);
}

static double bvp_psi(const orc_branching* B, int d, const double* x) {
  double xs[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k = 0; k < d; ++k) xs[k] = x[k];
  return orc_fun_eval(&B->psi, xs);
}

/* one tree; P[i] receives the value at output time i.  Returns 1 if pruned. */
static int bvp_tree_once(const orc_branching* B, const orc_branch_boundary* Bd, const double* x0,
                         const uint32_t key[2], int layout, int attempt, uint32_t tree, uint32_t point,
                         br_seg* stack, double* P, int64_t* segs_out, int64_t* substeps) {
  const int d = B->dim, nt = Bd->n_times;
  const double* tt = Bd->times;
  const double tend = tt[nt - 1];
  const int bounded = Bd->dom.kind != ORC_FREE;
  const uint64_t base = (uint64_t)label_base(B);
  int64_t segs = 0;
  for (int i = 0; i < nt; ++i) P[i] = 1.0;
  double x[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < d; ++k) x[k] = x0[k];
  if (!bounded || orc_inside(&Bd->dom, x))
    for (int i = 0; i < nt; ++i)
      if (tt[i] <= 0.0) P[i] *= bvp_psi(B, d, x);
  int top = 0;
  stack[0].label = 1;
  for (int k = 0; k < 3; ++k) stack[0].x[k] = x[k];
  stack[0].t = 0.0;
  top = 1;
  while (top > 0) {
    br_seg sg = stack[--top];
    segs += 1;
    if (segs > B->max_segments) { *segs_out = segs; return 1; }
    if (bounded && !orc_inside(&Bd->dom, sg.x)) {
      /* born outside (the start point, or the death point of its parent):
         stopped at its birth time */
      double xp[3];
      orc_project(&Bd->dom, sg.x, xp);
      for (int i = 0; i < nt; ++i)
        if (tt[i] >= sg.t) P[i] *= bvp_g(Bd, d, xp, tt[i] - sg.t);
      continue;
    }
    double ulife, utype;
    branch_uniforms(key, layout, sg.label, attempt, tree, point, &ulife, &utype);
    const double E = -log(ulife) / B->beta;
    const double sdeath = sg.t + E;
    const double send = sdeath < tend ? sdeath : tend;
    double s = sg.t;
    int k = 0;
    while (k < nt && !(tt[k] > s)) ++k;
    uint64_t gi = 0;
    int stopped = 0;
    while (s < send) {
      double sn = s + Bd->dt;
      if (send < sn) sn = send;
      if (k < nt && tt[k] < sn) sn = tt[k];
      const double sd = B->sigma * sqrt(sn - s);
      *substeps += 1;
      for (int c = 0; c < d; ++c) {
        const double z = bvp_normal(key, layout, sg.label, attempt, tree, point, gi++);
        sg.x[c] = sg.x[c] + sd * z;
      }
      s = sn;
      /* the sub-step that ends at the particle's death is followed by the
         branching, not by the boundary test: its children start there and
         are tested at their birth */
      const int dies = s == sdeath && sdeath < tend;
      const int out = bounded && (Bd->boundary_shift > 0.0 ? !inside_shrunk(&Bd->dom, sg.x, Bd->boundary_shift * sd)
                                                            : !orc_inside(&Bd->dom, sg.x));
      if (!dies && out) {
        double xp[3];
        orc_project(&Bd->dom, sg.x, xp);
        for (int i = 0; i < nt; ++i)
          if (tt[i] >= s) P[i] *= bvp_g(Bd, d, xp, tt[i] - s);
        stopped = 1;
        break;
      }
      if (k < nt && s == tt[k]) {
        P[k] *= bvp_psi(B, d, sg.x);
        ++k;
      }
    }
    if (stopped || !(sdeath < tend)) continue;
    const int I = pick_type(B->q, utype);
    const double wmark = B->alpha[I] / B->q[I];
    for (int i = 0; i < nt; ++i)
      if (tt[i] > sdeath) P[i] *= wmark;
    for (int i = I - 1; i >= 0; --i) {
      uint64_t child = base * sg.label + (uint64_t)i;
      if (child >= (1ull << 48) || sg.label >= (1ull << 47) || top >= BR_MAX_STACK) { *segs_out = segs; return 1; }
      stack[top].label = child;
      for (int c = 0; c < 3; ++c) stack[top].x[c] = sg.x[c];
      stack[top].t = sdeath;
      top++;
    }
  }
  *segs_out = segs;
  return 0;
}

typedef struct {
  const orc_branching* B;
  const orc_branch_boundary* Bd;
  const double* points;
  int64_t n_points, trees;
  uint32_t key[2];
  int layout;
  orc_stat* out;
  double* dump_val;
  int64_t* dump_segs;
  int64_t* redrawn_per_point;
} bvp_ctx;

static void bvp_point(void* vctx, int64_t i, int worker) {
  (void)worker;
  bvp_ctx* C = (bvp_ctx*)vctx;
  const int nt = C->Bd->n_times, d = C->B->dim;
  br_seg* stack = (br_seg*)malloc(sizeof(br_seg) * BR_MAX_STACK);
  double* P = (double*)malloc(sizeof(double) * (size_t)nt);
  orc_stat* s = (orc_stat*)calloc((size_t)nt, sizeof(orc_stat));
  int64_t redrawn = 0, subsum = 0, cens = 0;
  for (int64_t t = 0; t < C->trees; ++t) {
    int64_t segs = 0;
    int ok = 0;
    for (int attempt = 0; attempt < 16; ++attempt) {
      if (bvp_tree_once(C->B, C->Bd, &C->points[i * d], C->key, C->layout, attempt, (uint32_t)t, (uint32_t)i,
                        stack, P, &segs, &subsum) == 0) { ok = 1; break; }
      redrawn += 1;
    }
    if (!ok) {
      for (int k = 0; k < nt; ++k) P[k] = 0.0;
      cens += 1;
    }
    for (int k = 0; k < nt; ++k) welford_push(&s[k], P[k]);
    if (C->dump_val)
      for (int k = 0; k < nt; ++k) C->dump_val[(i * C->trees + t) * nt + k] = P[k];
    if (C->dump_segs) C->dump_segs[i * C->trees + t] = segs;
  }
  for (int k = 0; k < nt; ++k) {
    s[k].steps = subsum;
    s[k].censored = cens;
    C->out[(int64_t)k * C->n_points + i] = s[k];
  }
  C->redrawn_per_point[i] = redrawn;
  free(s); free(P); free(stack);
}

int orc_branching_bvp(const orc_branching* B, const orc_branch_boundary* Bd, const double* points,
                      int64_t n_points, int64_t trees, uint64_t seed, int layout, int n_threads,
                      orc_stat* out, double* dump_val, int64_t* dump_segs, int64_t* redrawn) {
  if (B->dim < 1 || B->dim > 3 || !(B->beta > 0.0) || Bd->n_times < 1 || !(Bd->dt > 0.0)) return -1;
  if (Bd->dom.kind != ORC_FREE && Bd->dom.dim != B->dim) return -1;
  for (int i = 0; i < Bd->n_times; ++i)
    if (!(Bd->times[i] >= 0.0) || (i > 0 && !(Bd->times[i] > Bd->times[i - 1]))) return -1;
  if (n_points >= (1ll << 24)) return -1;
  /* Gaussian blocks per particle stay below 2^16 */
  const double per = layout == ORC_QUAD24 ? 4.0 : 2.0;
  if ((ceil(Bd->times[Bd->n_times - 1] / Bd->dt) + Bd->n_times + 2.0) * B->dim / per >= 65536.0) return -1;
  bvp_ctx C;
  memset(&C, 0, sizeof(C));
  C.B = B; C.Bd = Bd; C.points = points; C.n_points = n_points; C.trees = trees; C.layout = layout;
  C.out = out; C.dump_val = dump_val; C.dump_segs = dump_segs;
  C.redrawn_per_point = (int64_t*)calloc((size_t)n_points + 1, sizeof(int64_t));
  make_key(seed, C.key);
  run_pool(n_threads, n_points, bvp_point, &C);
  int64_t tot = 0;
  for (int64_t i = 0; i < n_points; ++i) tot += C.redrawn_per_point[i];
  if (redrawn) *redrawn = tot;
  free(C.redrawn_per_point);
  return 0;
}
