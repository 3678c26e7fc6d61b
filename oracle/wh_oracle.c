/*
 * Plain double-precision CPU oracle for the explicit WaveHoltz iteration.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
 * the CPU-baseline leg of the benchmark may load this code.  The GPU library
 * never links, includes or calls it, and it shares no source with the library.
 *
 * What it computes (Appelo, Banks, Henshaw, Schwendeman, "An optimal O(N)
 * Helmholtz solver for complex geometry using WaveHoltz and overset grids"):
 *   - the p-th order Cartesian approximation L_ph = c^2 * Delta_{h,p} of
 *     Sec. 3.1 and the b_mu theorem of Sec. 6.1 (eq. SecondDerivOrderp truncated as in
 *     Appendix B, eq. HelmholtzOrderp): sum over mu < p/2 of
 *     b_mu (-h^2 D+D-)^mu D+D-, with b_mu = 2 (mu!)^2 / (2mu+2)!;
 *   - homogeneous Dirichlet walls of the unit box; ghost values outside a wall
 *     follow the odd reflection u(-j) = -u(j) (the paper leaves the high-order
 *     closure to its references; odd reflection is the reading used here);
 *   - the explicit scheme eq. (WaveSchemeexplicit) with forcing
 *     -f cos(omega_e t^n), the first step obtained by eliminating W^{-1} with
 *     the zero initial velocity (Sec. 4.2.1);
 *   - the trapezoid-rule time filter eq. (updateDiscreteExplicit) with
 *     sigma_0 = sigma_N = 1/2, normalised by the filter length Tbar = Np*T~.
 *
 * Everything is written as plain loops in the order the paper states the
 * steps: no blocking, no fusion.  The spacing h is passed explicitly so the
 * same routine can run on a sub-box of a larger grid (used to compute single
 * sampled outputs of a large apply through their domain of dependence).
 *
 * Layout: node arrays of (n_z+1)(n_y+1)(n_x+1) doubles, x fastest.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_HALF 4 /* supports orders p = 2, 4, 6, 8 */

/* eq. (uxxCoeff), Sec. 6.1: b_mu = 2 (mu!)^2 / (2 mu + 2)! */
double orc_b_mu(int mu) {
  double num = 2.0, den = 1.0;
  for (int k = 1; k <= mu; ++k) num *= (double)k * (double)k;
  for (int k = 1; k <= 2 * mu + 2; ++k) den *= (double)k;
  return num / den;
}

typedef struct {
  int dim;
  int64_t n[3];   /* cells per axis; nodes 0..n[m] */
  double h[3];    /* spacing per axis */
  int order;      /* p */
} orc_grid;

static int64_t orc_nodes(const orc_grid *g) {
  int64_t t = 1;
  for (int m = 0; m < g->dim; ++m) t *= (g->n[m] + 1);
  return t;
}

static int64_t orc_index(const orc_grid *g, const int64_t ix[3]) {
  int64_t idx = 0;
  for (int m = g->dim - 1; m >= 0; --m) idx = idx * (g->n[m] + 1) + ix[m];
  return idx;
}

static int orc_is_boundary(const orc_grid *g, const int64_t ix[3]) {
  for (int m = 0; m < g->dim; ++m)
    if (ix[m] == 0 || ix[m] == g->n[m]) return 1;
  return 0;
}

/* Value of W at a node that may lie outside the box: odd reflection about the
 * wall that was crossed (u(-j) = -u(j), u(n+j) = -u(n-j)). */
static double orc_value(const orc_grid *g, const double *W, const int64_t ix_in[3]) {
  int64_t ix[3] = {ix_in[0], ix_in[1], ix_in[2]};
  double sign = 1.0;
  for (int m = 0; m < g->dim; ++m) {
    if (ix[m] < 0) {
      ix[m] = -ix[m];
      sign = -sign;
    } else if (ix[m] > g->n[m]) {
      ix[m] = 2 * g->n[m] - ix[m];
      sign = -sign;
    }
  }
  return sign * W[orc_index(g, ix)];
}

/* d^2/dx_m^2 at node ix by sum_{mu<p/2} b_mu (-h^2)^mu (D+D-)^{mu+1}: the
 * line segment through ix along axis m is differenced repeatedly. */
static double orc_second_derivative(const orc_grid *g, const double *W, const int64_t ix[3], int m) {
  const int r = g->order / 2;
  double seg[2 * ORC_MAX_HALF + 1];
  int64_t jx[3] = {ix[0], ix[1], ix[2]};
  for (int s = -r; s <= r; ++s) {
    jx[m] = ix[m] + s;
    seg[s + r] = orc_value(g, W, jx);
  }
  const double h2 = g->h[m] * g->h[m];
  double result = 0.0;
  double scale = 1.0; /* (-h^2)^mu */
  int len = 2 * r + 1;
  for (int mu = 0; mu < r; ++mu) {
    /* one more application of D+D- shrinks the segment by one node per side */
    for (int s = 0; s + 2 < len; ++s) seg[s] = (seg[s + 2] - 2.0 * seg[s + 1] + seg[s]) / h2;
    len -= 2;
    result += orc_b_mu(mu) * scale * seg[len / 2];
    scale *= -h2;
  }
  return result;
}

/* out = L_ph W = c^2 * Delta_{h,p} W at interior nodes; 0 on the walls. */
static void orc_apply_L(const orc_grid *g, const double *c2, const double *W, double *out) {
  const int64_t total = orc_nodes(g);
#pragma omp parallel for schedule(static)
  for (int64_t idx = 0; idx < total; ++idx) {
    int64_t ix[3] = {0, 0, 0}, rem = idx;
    for (int m = 0; m < g->dim; ++m) {
      ix[m] = rem % (g->n[m] + 1);
      rem /= (g->n[m] + 1);
    }
    if (orc_is_boundary(g, ix)) {
      out[idx] = 0.0;
      continue;
    }
    double lap = 0.0;
    for (int m = 0; m < g->dim; ++m) lap += orc_second_derivative(g, W, ix, m);
    out[idx] = c2[idx] * lap;
  }
}

static int orc_make_grid(orc_grid *g, int dim, const int64_t *n, const double *h, int order) {
  if (dim < 1 || dim > 3) return -1;
  if (order < 2 || order > 2 * ORC_MAX_HALF || (order % 2) != 0) return -1;
  g->dim = dim;
  g->order = order;
  for (int m = 0; m < 3; ++m) {
    g->n[m] = (m < dim) ? n[m] : 0;
    g->h[m] = (m < dim) ? h[m] : 1.0;
    if (m < dim && (n[m] < 2 || !(h[m] > 0.0))) return -1;
  }
  return 0;
}

/* Number of nodes of a grid, exported for the Python side. */
int64_t orc_node_count(int dim, const int64_t *n) {
  int64_t t = 1;
  for (int m = 0; m < dim; ++m) t *= (n[m] + 1);
  return t;
}

/* out = L_ph W (exported so tests can check the operator by itself). */
int orc_laplacian(int dim, const int64_t *n, const double *h, int order, const double *c2,
                  const double *W, double *out) {
  orc_grid g;
  if (orc_make_grid(&g, dim, n, h, order)) return -1;
  orc_apply_L(&g, c2, W, out);
  return 0;
}

/* Trapezoid filter weight of time level n (eq. updateDiscreteExplicit over
 * Tbar = Np * 2pi/omega_e):  (2/Tbar) sigma_n dt (cos(omega_e t^n) - alpha/2). */
double orc_filter_weight(int64_t n, int64_t nsteps, double dt, double omega_e, double alpha) {
  const double Tbar = (double)nsteps * dt; /* Np periods of length Nt*dt */
  const double sigma = (n == 0 || n == nsteps) ? 0.5 : 1.0;
  const double tn = (double)n * dt;
  return (2.0 / Tbar) * sigma * dt * (cos(omega_e * tn) - 0.5 * alpha);
}

/*
 * One WaveHoltz application (Alg. 1, one pass of the loop body):
 *   W^0 = v, zero initial velocity, Np periods of Nt leapfrog steps with
 *   forcing -s f cos(omega_e t^n) (s = with_forcing), and the filtered result
 *   filtered = (2/Tbar) sum_n sigma_n dt (cos(omega_e t^n) - alpha/2) W^n.
 * Values of v and f on wall nodes are ignored (treated as 0).
 * w_final (nullable) receives W^{Np*Nt}.
 */
int orc_apply(int dim, const int64_t *n, const double *h, int order, const double *c2,
              const double *f, const double *v, int64_t nt, int64_t periods, double dt,
              double omega_e, double alpha, int with_forcing, double *filtered, double *w_final) {
  orc_grid g;
  if (orc_make_grid(&g, dim, n, h, order)) return -1;
  if (nt < 1 || periods < 1 || !(dt > 0.0)) return -1;
  const int64_t total = orc_nodes(&g);
  const int64_t nsteps = nt * periods;
  const double s = with_forcing ? 1.0 : 0.0;

  double *Wprev = (double *)calloc((size_t)total, sizeof(double));
  double *Wcur = (double *)calloc((size_t)total, sizeof(double));
  double *Wnext = (double *)calloc((size_t)total, sizeof(double));
  double *LW = (double *)calloc((size_t)total, sizeof(double));
  double *fint = (double *)calloc((size_t)total, sizeof(double));
  if (!Wprev || !Wcur || !Wnext || !LW || !fint) {
    free(Wprev); free(Wcur); free(Wnext); free(LW); free(fint);
    return -2;
  }

  /* W^0 = v on interior nodes, 0 on the walls; f likewise. */
  for (int64_t idx = 0; idx < total; ++idx) {
    int64_t ix[3] = {0, 0, 0}, rem = idx;
    for (int m = 0; m < dim; ++m) {
      ix[m] = rem % (n[m] + 1);
      rem /= (n[m] + 1);
    }
    const int wall = orc_is_boundary(&g, ix);
    Wcur[idx] = wall ? 0.0 : v[idx];
    fint[idx] = wall ? 0.0 : (f ? f[idx] : 0.0);
  }

  /* filter term of level 0 */
  {
    const double w0 = orc_filter_weight(0, nsteps, dt, omega_e, alpha);
    for (int64_t idx = 0; idx < total; ++idx) filtered[idx] = w0 * Wcur[idx];
  }

  /* first step: W^1 = W^0 + dt^2/2 (L W^0 - s f cos(0)) */
  orc_apply_L(&g, c2, Wcur, LW);
  for (int64_t idx = 0; idx < total; ++idx)
    Wnext[idx] = Wcur[idx] + 0.5 * dt * dt * (LW[idx] - s * fint[idx]);
  {
    double *t = Wprev; Wprev = Wcur; Wcur = Wnext; Wnext = t;
    const double w1 = orc_filter_weight(1, nsteps, dt, omega_e, alpha);
    for (int64_t idx = 0; idx < total; ++idx) filtered[idx] += w1 * Wcur[idx];
  }

  /* leapfrog: W^{n+1} = 2 W^n - W^{n-1} + dt^2 (L W^n - s f cos(omega_e t^n)) */
  for (int64_t step = 1; step < nsteps; ++step) {
    const double tn = (double)step * dt;
    const double forcing = s * cos(omega_e * tn);
    orc_apply_L(&g, c2, Wcur, LW);
#pragma omp parallel for schedule(static)
    for (int64_t idx = 0; idx < total; ++idx)
      Wnext[idx] = 2.0 * Wcur[idx] - Wprev[idx] + dt * dt * (LW[idx] - forcing * fint[idx]);
    double *t = Wprev; Wprev = Wcur; Wcur = Wnext; Wnext = t;
    const double wn = orc_filter_weight(step + 1, nsteps, dt, omega_e, alpha);
#pragma omp parallel for schedule(static)
    for (int64_t idx = 0; idx < total; ++idx) filtered[idx] += wn * Wcur[idx];
  }

  if (w_final) memcpy(w_final, Wcur, (size_t)total * sizeof(double));
  free(Wprev); free(Wcur); free(Wnext); free(LW); free(fint);
  return 0;
}

/* Residual of the discrete Helmholtz problem (eq. HelmholtzDiscrete with the
 * sign convention of eq. HelmholtzBVP): res = L_ph u + omega^2 u - f on
 * interior nodes, 0 on the walls. */
int orc_helmholtz_residual(int dim, const int64_t *n, const double *h, int order, const double *c2,
                           const double *f, const double *u, double omega, double *res) {
  orc_grid g;
  if (orc_make_grid(&g, dim, n, h, order)) return -1;
  const int64_t total = orc_nodes(&g);
  orc_apply_L(&g, c2, u, res);
  for (int64_t idx = 0; idx < total; ++idx) {
    int64_t ix[3] = {0, 0, 0}, rem = idx;
    for (int m = 0; m < dim; ++m) {
      ix[m] = rem % (n[m] + 1);
      rem /= (n[m] + 1);
    }
    res[idx] = orc_is_boundary(&g, ix) ? 0.0 : res[idx] + omega * omega * u[idx] - f[idx];
  }
  return 0;
}

/* Number of threads OpenMP would use (1 when built without OpenMP). */
int orc_max_threads(void) {
#ifdef _OPENMP
  extern int omp_get_max_threads(void);
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads of the following parallel regions (timing only; no effect when
 * built without OpenMP or for n < 1). */
void orc_set_threads(int n) {
#ifdef _OPENMP
  extern void omp_set_num_threads(int);
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
