/* Small end-to-end run of the oracle for the host-sanitizer test: a walk with
 * drift, killing, source and terms, its adjoint, Walk on Spheres, the
 * branching estimator and the branching estimator with a boundary, all on a
 * thread pool of 4 workers.  Exit status 0 when every call succeeds. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "oracle.h"

int main(void) {
  orc_factor fac[4];
  memset(fac, 0, sizeof fac);
  fac[0].fn = ORC_SIN; fac[0].dim = 1; fac[0].power = 1; fac[0].a = 3.14159;
  fac[1].fn = ORC_COS; fac[1].dim = 0; fac[1].power = 1; fac[1].a = 1.0;
  fac[2].fn = ORC_EXP; fac[2].dim = 1; fac[2].power = 1; fac[2].a = 1.0;
  fac[3].fn = ORC_TANH; fac[3].dim = 2; fac[3].power = 1; fac[3].a = 0.5;   /* time argument of g (dim 2) */
  double coef[4] = {0.3, 0.2, 0.5, -0.4};
  int32_t mexp[3] = {0, 0, 0};
  double mcoef[1] = {1.0};
  orc_linear L;
  memset(&L, 0, sizeof L);
  L.dom.kind = ORC_BALL; L.dom.dim = 2; L.dom.radius = 1.0;
  L.sigma = 1.0;
  L.b[0] = (orc_fun){1, 1, &fac[0], &coef[0], 0, 0, mexp, mcoef};
  L.c = (orc_fun){0, 0, NULL, NULL, 1, 0, mexp, mcoef};
  L.f = (orc_fun){1, 1, &fac[1], &coef[1], 0, 0, mexp, mcoef};
  L.g = (orc_fun){1, 1, &fac[2], &coef[2], 0, 0, mexp, mcoef};
  double nodes[6] = {0.1, 0.2, -0.3, 0.4, 0.5, -0.5};
  int64_t paths[3] = {500, 300, 700};
  orc_stat st[16];
  int rc = orc_walk(&L, nodes, 3, paths, 1e-2, 7, ORC_PAIR52, 2000, 4, st, NULL, NULL, NULL);
  double w[3] = {1.0, -0.5, 2.0}, dg[1] = {0}, df[1] = {0}, dc[1] = {0}, dgm[1] = {0}, dfm[1] = {0}, dcm[1] = {0};
  rc |= orc_walk_adjoint(&L, nodes, 3, paths, 1e-2, 7, ORC_QUAD24, 2000, 4, w, dg, dgm, df, dfm, dc, dcm, st);
  orc_linear H = L;
  H.b[0] = (orc_fun){0, 0, NULL, NULL, 0, 0, mexp, mcoef};
  H.c = H.b[0];
  H.f = H.b[0];
  rc |= orc_wos(&H, nodes, 3, paths, 1e-3, 7, ORC_PAIR52, 100000, 4, st, NULL, NULL, NULL);
  orc_branching B;
  memset(&B, 0, sizeof B);
  B.dim = 2; B.max_segments = 64; B.sigma = 1.0; B.beta = 1.0; B.T = 0.7;
  B.alpha[2] = 1.0; B.q[2] = 1.0;
  double c3 = 0.3;
  B.psi = (orc_fun){0, 0, NULL, NULL, 1, 0, mexp, &c3};
  int64_t red = 0;
  rc |= orc_branching_dfs(&B, nodes, 3, 400, 5, ORC_QUAD24, 4, st, NULL, NULL, &red);
  orc_branch_boundary Bd;
  memset(&Bd, 0, sizeof Bd);
  Bd.dom = L.dom;
  Bd.g = (orc_fun){1, 1, &fac[3], &coef[3], 0, 0, mexp, mcoef};
  double times[3] = {0.0, 0.3, 0.7};
  Bd.dt = 0.01; Bd.n_times = 3; Bd.times = times; Bd.boundary_shift = 0.5826;
  rc |= orc_branching_bvp(&B, &Bd, nodes, 3, 400, 5, ORC_PAIR52, 4, st, NULL, NULL, &red);
  printf("rc %d mean %.6f\n", rc, st[0].mean);
  return rc != 0;
}
