/*
 * dbm_oracle.c -- plain FP64 CPU oracle of the multi-component D2V16 discrete
 * Boltzmann model of Lin, Luo, Fei and Succi (arXiv:2006.15932).
 *
 * TEST INFRASTRUCTURE ONLY.  It is the slow, obviously-correct statement of
 * what the GPU path computes, used by the tests, the package smoke check and
 * the benchmark's CPU-baseline leg.  It shares no code with the GPU library.
 *
 * Everything is FP64, built with -ffp-contract=off so that no multiply-add is
 * fused.  The steps follow the paper's order:
 *   velocity set (Eq.15) -> moment matrix M (rows listed after Eq.14) ->
 *   M^{-1} by Gauss-Jordan elimination with partial pivoting ->
 *   per cell: moments (conservation statement under Eq.6, Eqs.8-10) ->
 *   reaction (Eqs.1-2 and Eq.5) -> force (Eq.6) -> f^eq = M^{-1} fhat (Eq.16)
 *   -> BGK source (Eq.4) -> convection by the NND upwind scheme ->
 *   forward Euler (the paper's time scheme) or third-order TVD Runge-Kutta.
 *
 * Readings of points the paper leaves open (each one is a documented choice):
 *   - M row 9 is (v^2+eta^2) v_y; the printed v_x repeats row 8 and makes M
 *     singular, while fhat_9 carries u_y.
 *   - Eq.(13) is taken with the mixture T, the argument of f^eq, as in fhat.
 *   - Mixture u = sum m j / rho; T = (sum m E - rho u^2) / sum (D+I) n, which is
 *     what exact conservation of momentum and energy by Eq.(4) requires.
 *   - Reaction: extent xi = omega*tau (clamped so no reactant goes negative),
 *     n* = n + a xi, and T* from sum (D+I) n* T* = sum (D+I) n T + 2 Q xi.
 *   - Force: u_dagger = u^s + tau a, T_dagger = T^s - m tau^2 |a|^2/(D+I)
 *     (the choice that reproduces the momentum and energy sources of the
 *     modified NS equations exactly), or T_dagger = T^s.
 *   - NND interface value: f_j + minmod(f_j-f_{j-1}, f_{j+1}-f_j)/2 for a
 *     positive velocity component and its mirror image for a negative one.
 */
#include "dbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NV OR_NV
#define DIM 2.0

struct or_model {
  or_config cfg;
  or_species sp[OR_MAXS];
  or_reaction_step chem[OR_MAXR];
  double vx[OR_MAXS][NV], vy[OR_MAXS][NV], eta[OR_MAXS][NV], q[OR_MAXS][NV];
  double M[OR_MAXS][NV * NV], Minv[OR_MAXS][NV * NV];
  int mirx[OR_MAXS][NV], miry[OR_MAXS][NV];
};

static int g_threads = 1;

void or_set_threads(int n) { g_threads = n < 1 ? 1 : n; }
int or_get_threads(void) { return g_threads; }

/* ---------------------------------------------------------------------------
 * Velocity set, Eq.(15): four groups of four.  Groups a and c lie on the axes,
 * v(+-1,0) and its cyclic permutation; groups b and d on the diagonals,
 * v(+-1,+-1).  Order inside a group: counter-clockwise starting at +x (axes)
 * or at (+1,+1) (diagonals).  Each group carries its own eta.
 * ------------------------------------------------------------------------- */
static void velocity_set(const or_species *s, double *vx, double *vy, double *eta) {
  static const double axis[4][2] = {{1, 0}, {0, 1}, {-1, 0}, {0, -1}};
  static const double diag[4][2] = {{1, 1}, {-1, 1}, {-1, -1}, {1, -1}};
  for (int g = 0; g < 4; ++g) {
    for (int k = 0; k < 4; ++k) {
      int i = 4 * g + k;
      const double *d = (g % 2 == 0) ? axis[k] : diag[k];
      vx[i] = s->v[g] * d[0];
      vy[i] = s->v[g] * d[1];
      eta[i] = s->eta[g];
    }
  }
}

/* Moment matrix: the 16 rows listed after Eq.(14), M[r*16+i] = phi_r(v_i). */
static void moment_matrix(const double *vx, const double *vy, const double *eta,
                          double *M) {
  for (int i = 0; i < NV; ++i) {
    double x = vx[i], y = vy[i];
    double q = x * x + y * y + eta[i] * eta[i];
    M[0 * NV + i] = 1.0;
    M[1 * NV + i] = x;
    M[2 * NV + i] = y;
    M[3 * NV + i] = q;
    M[4 * NV + i] = x * x;
    M[5 * NV + i] = x * y;
    M[6 * NV + i] = y * y;
    M[7 * NV + i] = q * x;
    M[8 * NV + i] = q * y;
    M[9 * NV + i] = x * x * x;
    M[10 * NV + i] = x * x * y;
    M[11 * NV + i] = x * y * y;
    M[12 * NV + i] = y * y * y;
    M[13 * NV + i] = q * x * x;
    M[14 * NV + i] = q * x * y;
    M[15 * NV + i] = q * y * y;
  }
}

/* Gauss-Jordan elimination with partial pivoting.  Returns 0, or -1 when a
 * pivot falls below 1e-12 of the largest entry of A (rank-deficient). */
static int invert(const double *A, double *Ainv, int n) {
  double *W = (double *)malloc(sizeof(double) * n * 2 * n);
  if (!W) return -1;
  double amax = 0.0;
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < n; ++c) {
      W[r * 2 * n + c] = A[r * n + c];
      W[r * 2 * n + n + c] = (r == c) ? 1.0 : 0.0;
      if (fabs(A[r * n + c]) > amax) amax = fabs(A[r * n + c]);
    }
  int rc = 0;
  for (int col = 0; col < n && rc == 0; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (fabs(W[r * 2 * n + col]) > fabs(W[piv * 2 * n + col])) piv = r;
    if (!(fabs(W[piv * 2 * n + col]) > 1e-12 * amax)) { rc = -1; break; }
    if (piv != col)
      for (int c = 0; c < 2 * n; ++c) {
        double t = W[col * 2 * n + c];
        W[col * 2 * n + c] = W[piv * 2 * n + c];
        W[piv * 2 * n + c] = t;
      }
    double p = W[col * 2 * n + col];
    for (int c = 0; c < 2 * n; ++c) W[col * 2 * n + c] /= p;
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      double fct = W[r * 2 * n + col];
      if (fct == 0.0) continue;
      for (int c = 0; c < 2 * n; ++c) W[r * 2 * n + c] -= fct * W[col * 2 * n + c];
    }
  }
  if (rc == 0)
    for (int r = 0; r < n; ++r)
      for (int c = 0; c < n; ++c) Ainv[r * n + c] = W[r * 2 * n + n + c];
  free(W);
  return rc;
}

static double norm1(const double *A, int n) {
  double best = 0.0;
  for (int c = 0; c < n; ++c) {
    double s = 0.0;
    for (int r = 0; r < n; ++r) s += fabs(A[r * n + c]);
    if (s > best) best = s;
  }
  return best;
}

/* Index of the velocity with one component reflected (specular wall). */
static int mirror_index(const double *vx, const double *vy, const double *eta, int i,
                        int flip_x) {
  double tx = flip_x ? -vx[i] : vx[i];
  double ty = flip_x ? vy[i] : -vy[i];
  for (int k = 0; k < NV; ++k)
    if (vx[k] == tx && vy[k] == ty && eta[k] == eta[i]) return k;
  return -1;
}

int or_create(const or_config *cfg, or_model **out) {
  if (!cfg || !out) return -1;
  *out = NULL;
  const or_config *c = cfg;
  if (c->nx < 1 || c->ny < 1 || !(c->dx > 0) || !(c->dy > 0) || !(c->dt > 0)) return -1;
  if (c->S < 1 || c->S > OR_MAXS || !c->sp) return -1;
  if (c->bc_x < 0 || c->bc_x > 2 || c->bc_y < 0 || c->bc_y > 2) return -1;
  if (c->scheme < 0 || c->scheme > 1 || c->limiter < 0 || c->limiter > 1) return -1;
  if (c->force_T_mode < 0 || c->force_T_mode > 1) return -1;
  for (int s = 0; s < c->S; ++s)
    if (!(c->sp[s].m > 0) || !(c->sp[s].tau > 0) || !(c->sp[s].I >= 0)) return -1;
  if (c->reaction_on) {
    if (c->fuel < 0 || c->fuel >= c->S || c->oxid < 0 || c->oxid >= c->S ||
        c->fuel == c->oxid)
      return -1;
    if (!(c->k_ov >= 0)) return -1;
    /* With species-dependent tau the post-reaction temperature is ambiguous. */
    for (int s = 1; s < c->S; ++s)
      if (c->sp[s].tau != c->sp[0].tau) return -5;
  }
  if (c->nchem < 0 || c->nchem > OR_MAXR || (c->nchem > 0 && !c->chem)) return -1;
  for (int r = 0; r < c->nchem; ++r) {
    const or_reaction_step *st = &c->chem[r];
    if (st->fuel < 0 || st->fuel >= c->S || st->oxid < 0 || st->oxid >= c->S) return -1;
    if (!(st->k >= 0) || !isfinite(st->k) || !isfinite(st->Ea_over_R) || !isfinite(st->Q))
      return -1;
    for (int s = 1; s < c->S; ++s)
      if (st->k > 0 && c->sp[s].tau != c->sp[0].tau) return -5;
  }
  or_model *md = (or_model *)calloc(1, sizeof(or_model));
  if (!md) return -1;
  md->cfg = *c;
  for (int s = 0; s < c->S; ++s) md->sp[s] = c->sp[s];
  md->cfg.sp = md->sp;
  for (int r = 0; r < c->nchem; ++r) md->chem[r] = c->chem[r];
  md->cfg.chem = c->nchem > 0 ? md->chem : NULL;
  for (int s = 0; s < c->S; ++s) {
    velocity_set(&md->sp[s], md->vx[s], md->vy[s], md->eta[s]);
    for (int i = 0; i < NV; ++i)
      md->q[s][i] = md->vx[s][i] * md->vx[s][i] + md->vy[s][i] * md->vy[s][i] +
                    md->eta[s][i] * md->eta[s][i];
    moment_matrix(md->vx[s], md->vy[s], md->eta[s], md->M[s]);
    if (invert(md->M[s], md->Minv[s], NV) != 0) { free(md); return -2; }
    double cond = norm1(md->M[s], NV) * norm1(md->Minv[s], NV);
    if (!(cond <= 1e12)) { free(md); return -2; }
    for (int i = 0; i < NV; ++i) {
      md->mirx[s][i] = mirror_index(md->vx[s], md->vy[s], md->eta[s], i, 1);
      md->miry[s][i] = mirror_index(md->vx[s], md->vy[s], md->eta[s], i, 0);
      if (md->mirx[s][i] < 0 || md->miry[s][i] < 0) { free(md); return -1; }
    }
  }
  *out = md;
  return 0;
}

void or_destroy(or_model *md) { free(md); }

int or_tables(const or_model *md, int s, double *vx, double *vy, double *eta, double *M,
              double *Minv) {
  if (!md || s < 0 || s >= md->cfg.S) return -1;
  for (int i = 0; i < NV; ++i) {
    if (vx) vx[i] = md->vx[s][i];
    if (vy) vy[i] = md->vy[s][i];
    if (eta) eta[i] = md->eta[s][i];
  }
  for (int k = 0; k < NV * NV; ++k) {
    if (M) M[k] = md->M[s][k];
    if (Minv) Minv[k] = md->Minv[s][k];
  }
  return 0;
}

/* ---------------------------------------------------------------------------
 * fhat^eq: the sixteen closed forms listed after Eq.(14), with theta = T/m and
 * K = D + I.  Components 10-13 use the same T as every other component.
 * ------------------------------------------------------------------------- */
void or_fhat(double n, double ux, double uy, double theta, double I, double *h) {
  double K = DIM + I;
  double u2 = ux * ux + uy * uy;
  double e2 = (K + 2.0) * theta + u2;
  double e4 = (K + 4.0) * theta + u2;
  h[0] = n;
  h[1] = n * ux;
  h[2] = n * uy;
  h[3] = n * (K * theta + u2);
  h[4] = n * (theta + ux * ux);
  h[5] = n * ux * uy;
  h[6] = n * (theta + uy * uy);
  h[7] = n * ux * e2;
  h[8] = n * uy * e2;
  h[9] = 3.0 * n * ux * theta + n * ux * ux * ux;
  h[10] = n * uy * theta + n * ux * ux * uy;
  h[11] = n * ux * theta + n * ux * uy * uy;
  h[12] = 3.0 * n * uy * theta + n * uy * uy * uy;
  h[13] = n * e2 * theta + n * ux * ux * e4;
  h[14] = n * ux * uy * e4;
  h[15] = n * e2 * theta + n * uy * uy * e4;
}

static void matvec(const double *A, const double *x, double *y) {
  for (int r = 0; r < NV; ++r) {
    double acc = 0.0;
    for (int c = 0; c < NV; ++c) acc += A[r * NV + c] * x[c];
    y[r] = acc;
  }
}

int or_feq(const or_model *md, int s, double n, double ux, double uy, double T,
           double *feq) {
  if (!md || s < 0 || s >= md->cfg.S) return -1;
  double h[NV];
  or_fhat(n, ux, uy, T / md->sp[s].m, md->sp[s].I, h);
  matvec(md->Minv[s], h, feq);
  return 0;
}

/* Per-species raw moments of one cell: n = sum f, j = sum f v, E = sum f q. */
static void species_moments(const or_model *md, int s, const double *f, double *n,
                            double *jx, double *jy, double *E) {
  double a = 0, b = 0, c = 0, d = 0;
  for (int i = 0; i < NV; ++i) {
    a += f[i];
    b += f[i] * md->vx[s][i];
    c += f[i] * md->vy[s][i];
    d += f[i] * md->q[s][i];
  }
  *n = a; *jx = b; *jy = c; *E = d;
}

/* Mixture velocity and temperature from the species moments. */
static void mixture(const or_model *md, const double *n, const double *jx,
                    const double *jy, const double *E, double *rho, double *ux,
                    double *uy, double *T) {
  double r = 0, px = 0, py = 0, e = 0, kn = 0;
  for (int s = 0; s < md->cfg.S; ++s) {
    double m = md->sp[s].m;
    r += m * n[s];
    px += m * jx[s];
    py += m * jy[s];
    e += m * E[s];
    kn += (DIM + md->sp[s].I) * n[s];
  }
  double u = px / r, v = py / r;
  *rho = r; *ux = u; *uy = v;
  *T = (e - r * (u * u + v * v)) / kn;
}

/* ---------------------------------------------------------------------------
 * Collision (Eq.4) + reaction (Eq.5) + force (Eq.6) of one cell.
 * src_i = [f^eq(n*,u,T*) - f_i]/tau
 *       + [f^eq(n,u_dagger,T_dagger) - f^eq(n,u^s,T^s)]/tau
 * ------------------------------------------------------------------------- */
int or_cell_source(const or_model *md, const double *fc, double *src) {
  const or_config *c = &md->cfg;
  const int S = c->S;
  double n[OR_MAXS] = {0}, jx[OR_MAXS] = {0}, jy[OR_MAXS] = {0}, E[OR_MAXS] = {0};
  double ns[OR_MAXS] = {0};
  for (int s = 0; s < S; ++s) species_moments(md, s, fc + s * NV, &n[s], &jx[s], &jy[s], &E[s]);
  double rho, ux, uy, T;
  mixture(md, n, jx, jy, E, &rho, &ux, &uy, &T);

  /* Chemical reaction, Eqs.(1)-(2): each step r has the rate
   * omega_r = k_r n^F n^O e^{-Ea_r/RT} and the extent xi_r = omega_r tau
   * within the relaxation time; the one-step reaction is the mechanism with
   * one step and the species' own coefficients.  If some reactant would be
   * consumed beyond its density, every extent is scaled by one common
   * factor.  Then n* = n + sum_r a_r xi_r and the energy balance
   * sum (D+I) n* T* = sum (D+I) n T + 2 sum_r Q_r xi_r gives T*. */
  double Ts = T;
  for (int s = 0; s < S; ++s) ns[s] = n[s];
  or_reaction_step one;
  const or_reaction_step *steps = c->chem;
  int nr = c->nchem;
  if (nr == 0 && c->reaction_on) {
    one.fuel = c->fuel; one.oxid = c->oxid;
    one.k = c->k_ov; one.Ea_over_R = c->Ea_over_R; one.Q = c->Q;
    for (int s = 0; s < S; ++s) one.a[s] = md->sp[s].a;
    steps = &one;
    nr = 1;
  }
  if (nr > 0) {
    double xi[OR_MAXR];
    for (int r = 0; r < nr; ++r) {
      double nF = n[steps[r].fuel] > 0 ? n[steps[r].fuel] : 0.0;
      double nO = n[steps[r].oxid] > 0 ? n[steps[r].oxid] : 0.0;
      xi[r] = steps[r].k * nF * nO * exp(-steps[r].Ea_over_R / T) * md->sp[0].tau;
    }
    double scale = 1.0;
    for (int s = 0; s < S; ++s) {
      double use = 0.0;
      for (int r = 0; r < nr; ++r)
        if (steps[r].a[s] < 0) use += -steps[r].a[s] * xi[r];
      double avail = n[s] > 0 ? n[s] : 0.0;
      if (use > avail && avail / use < scale) scale = avail / use;
    }
    double heat = 0.0, kn = 0, kns = 0;
    for (int r = 0; r < nr; ++r) {
      xi[r] *= scale;
      heat += 2.0 * steps[r].Q * xi[r];
      for (int s = 0; s < S; ++s) ns[s] += steps[r].a[s] * xi[r];
    }
    for (int s = 0; s < S; ++s) {
      kn += (DIM + md->sp[s].I) * n[s];
      kns += (DIM + md->sp[s].I) * ns[s];
    }
    Ts = (T * kn + heat) / kns;
  }

  const int force_on = (c->ax != 0.0 || c->ay != 0.0);
  for (int s = 0; s < S; ++s) {
    const double m = md->sp[s].m, I = md->sp[s].I, tau = md->sp[s].tau;
    const double K = DIM + I;
    double g[NV], h1[NV], h2[NV], feq[NV];
    or_fhat(ns[s], ux, uy, Ts / m, I, g);
    if (force_on && n[s] > 1e-300) {
      double us = jx[s] / n[s], vs = jy[s] / n[s];
      double Tsp = m * (E[s] / n[s] - us * us - vs * vs) / K;
      double ud = us + tau * c->ax, vd = vs + tau * c->ay;
      double Td = Tsp;
      if (c->force_T_mode == OR_FORCE_T_EXACT)
        Td = Tsp - m * tau * tau * (c->ax * c->ax + c->ay * c->ay) / K;
      or_fhat(n[s], ud, vd, Td / m, I, h1);
      or_fhat(n[s], us, vs, Tsp / m, I, h2);
      for (int k = 0; k < NV; ++k) g[k] += h1[k] - h2[k];
    }
    matvec(md->Minv[s], g, feq);
    for (int i = 0; i < NV; ++i) src[s * NV + i] = (feq[i] - fc[s * NV + i]) / tau;
  }
  return 0;
}

/* ---------------------------------------------------------------------------
 * Boundary index map for one axis.  Returns the interior index and toggles
 * *flip once per specular reflection.
 * ------------------------------------------------------------------------- */
static int bc_map(int j, int n, int bc, int *flip) {
  if (j >= 0 && j < n) return j;
  if (bc == OR_BC_PERIODIC) return ((j % n) + n) % n;
  if (bc == OR_BC_OUTFLOW) return j < 0 ? 0 : n - 1;
  while (j < 0 || j >= n) { /* wall: reflect about the boundary face */
    j = (j < 0) ? (-1 - j) : (2 * n - 1 - j);
    *flip ^= 1;
  }
  return j;
}

static double minmod(double a, double b) {
  if (a > 0 && b > 0) return a < b ? a : b;
  if (a < 0 && b < 0) return a > b ? a : b;
  return 0.0;
}

/* Interface value between j and j+1 from f_{j-1}, f_j, f_{j+1}, f_{j+2}. */
static double face(double fm1, double f0, double fp1, double fp2, double c, int lim) {
  if (c > 0) {
    double slope = (lim == OR_LIM_MINMOD) ? minmod(f0 - fm1, fp1 - f0) : (f0 - fm1);
    return f0 + 0.5 * slope;
  }
  double slope = (lim == OR_LIM_MINMOD) ? minmod(fp1 - f0, fp2 - fp1) : (fp2 - fp1);
  return fp1 - 0.5 * slope;
}

/* Convection -v.grad f of every plane, on a copy padded by two ghost cells. */
static void convection(const or_model *md, const double *f, double *C) {
  const or_config *c = &md->cfg;
  const int nx = c->nx, ny = c->ny, S = c->S;
  const int px = nx + 4, py = ny + 4;
  const size_t plane = (size_t)nx * ny;
#pragma omp parallel num_threads(g_threads)
  {
    double *P = (double *)malloc(sizeof(double) * (size_t)px * py);
#pragma omp for schedule(static)
    for (int si = 0; si < S * NV; ++si) {
      const int s = si / NV, i = si % NV;
      for (int yy = -2; yy < ny + 2; ++yy) {
        for (int xx = -2; xx < nx + 2; ++xx) {
          int fx = 0, fy = 0;
          int sx = bc_map(xx, nx, c->bc_x, &fx);
          int sy = bc_map(yy, ny, c->bc_y, &fy);
          int p = i;
          if (fx) p = md->mirx[s][p];
          if (fy) p = md->miry[s][p];
          P[(size_t)(yy + 2) * px + (xx + 2)] =
              f[((size_t)s * NV + p) * plane + (size_t)sy * nx + sx];
        }
      }
      const double vx = md->vx[s][i], vy = md->vy[s][i];
      for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
          const double *r = P + (size_t)(y + 2) * px + (x + 2);
          double dfx = 0.0, dfy = 0.0;
          if (vx != 0.0) {
            double fr = face(r[-1], r[0], r[1], r[2], vx, c->limiter);
            double fl = face(r[-2], r[-1], r[0], r[1], vx, c->limiter);
            dfx = (fr - fl) / c->dx;
          }
          if (vy != 0.0) {
            double fr = face(r[-px], r[0], r[px], r[2 * px], vy, c->limiter);
            double fl = face(r[-2 * px], r[-px], r[0], r[px], vy, c->limiter);
            dfy = (fr - fl) / c->dy;
          }
          C[((size_t)s * NV + i) * plane + (size_t)y * nx + x] = -(vx * dfx + vy * dfy);
        }
      }
    }
    free(P);
  }
}

int or_rhs(const or_model *md, const double *f, double *L) {
  if (!md || !f || !L) return -1;
  const or_config *c = &md->cfg;
  const int nx = c->nx, ny = c->ny, S = c->S;
  const size_t plane = (size_t)nx * ny;
  convection(md, f, L);
#pragma omp parallel for num_threads(g_threads) schedule(static)
  for (int y = 0; y < ny; ++y) {
    double fc[OR_MAXS * NV], src[OR_MAXS * NV];
    for (int x = 0; x < nx; ++x) {
      size_t cell = (size_t)y * nx + x;
      for (int k = 0; k < S * NV; ++k) fc[k] = f[(size_t)k * plane + cell];
      or_cell_source(md, fc, src);
      for (int k = 0; k < S * NV; ++k) L[(size_t)k * plane + cell] += src[k];
    }
  }
  return 0;
}

/* One stage: out = alpha*fn + beta*(fs + dt*L(fs)). */
static void stage(const or_model *md, const double *fn, const double *fs, double *out,
                  double *L, double alpha, double beta) {
  const size_t tot = (size_t)md->cfg.S * NV * md->cfg.nx * md->cfg.ny;
  const double dt = md->cfg.dt;
  or_rhs(md, fs, L);
#pragma omp parallel for num_threads(g_threads) schedule(static)
  for (size_t k = 0; k < tot; ++k) {
    double adv = fs[k] + dt * L[k];
    out[k] = (alpha == 0.0) ? adv : alpha * fn[k] + beta * adv;
  }
}

int or_run(const or_model *md, double *f, int nsteps) {
  if (!md || !f || nsteps < 0) return -1;
  const size_t tot = (size_t)md->cfg.S * NV * md->cfg.nx * md->cfg.ny;
  double *L = (double *)malloc(sizeof(double) * tot);
  double *f1 = (double *)malloc(sizeof(double) * tot);
  double *f2 = (double *)malloc(sizeof(double) * tot);
  if (!L || !f1 || !f2) { free(L); free(f1); free(f2); return -1; }
  for (int n = 0; n < nsteps; ++n) {
    if (md->cfg.scheme == OR_EULER) {
      stage(md, f, f, f1, L, 0.0, 1.0);
      memcpy(f, f1, sizeof(double) * tot);
    } else { /* Shu-Osher TVD-RK3 */
      stage(md, f, f, f1, L, 0.0, 1.0);
      stage(md, f, f1, f2, L, 0.75, 0.25);
      stage(md, f, f2, f1, L, 1.0 / 3.0, 2.0 / 3.0);
      memcpy(f, f1, sizeof(double) * tot);
    }
  }
  free(L); free(f1); free(f2);
  return 0;
}

int or_init_equilibrium(const or_model *md, const double *n_sp, const double *ux,
                        const double *uy, const double *T, double *f) {
  if (!md || !n_sp || !ux || !uy || !T || !f) return -1;
  const int S = md->cfg.S;
  const size_t plane = (size_t)md->cfg.nx * md->cfg.ny;
#pragma omp parallel for num_threads(g_threads) schedule(static)
  for (size_t cell = 0; cell < plane; ++cell) {
    double feq[NV];
    for (int s = 0; s < S; ++s) {
      or_feq(md, s, n_sp[(size_t)s * plane + cell], ux[cell], uy[cell], T[cell], feq);
      for (int i = 0; i < NV; ++i) f[((size_t)s * NV + i) * plane + cell] = feq[i];
    }
  }
  return 0;
}

int or_moments(const or_model *md, const double *f, double *rho_sp, double *ux,
               double *uy, double *T) {
  if (!md || !f) return -1;
  const int S = md->cfg.S;
  const size_t plane = (size_t)md->cfg.nx * md->cfg.ny;
#pragma omp parallel for num_threads(g_threads) schedule(static)
  for (size_t cell = 0; cell < plane; ++cell) {
    double fc[NV], n[OR_MAXS], jx[OR_MAXS], jy[OR_MAXS], E[OR_MAXS];
    for (int s = 0; s < S; ++s) {
      for (int i = 0; i < NV; ++i) fc[i] = f[((size_t)s * NV + i) * plane + cell];
      species_moments(md, s, fc, &n[s], &jx[s], &jy[s], &E[s]);
      if (rho_sp) rho_sp[(size_t)s * plane + cell] = md->sp[s].m * n[s];
    }
    double rho, u, v, t;
    mixture(md, n, jx, jy, E, &rho, &u, &v, &t);
    if (ux) ux[cell] = u;
    if (uy) uy[cell] = v;
    if (T) T[cell] = t;
  }
  return 0;
}

/* Eqs.(17)-(20): Delta = m sum_i (f_i - f_i^eq(n^s,u,T)) phi_i for the rows
 * v_x^2, v_xv_y, v_y^2 (Delta_2), q v_x, q v_y (Delta_3,1), v_x^3, v_x^2v_y,
 * v_xv_y^2, v_y^3 (Delta_3), q v_x^2, q v_xv_y, q v_y^2 (Delta_4,2). */
int or_noneq(const or_model *md, const double *f, double *delta, double *totals) {
  if (!md || !f) return -1;
  const or_config *c = &md->cfg;
  const int S = c->S;
  const size_t plane = (size_t)c->nx * c->ny;
  if (delta) {
#pragma omp parallel for num_threads(g_threads) schedule(static)
    for (size_t cell = 0; cell < plane; ++cell) {
      double fc[OR_MAXS][NV], n[OR_MAXS], jx[OR_MAXS], jy[OR_MAXS], E[OR_MAXS];
      for (int s = 0; s < S; ++s) {
        for (int i = 0; i < NV; ++i) fc[s][i] = f[((size_t)s * NV + i) * plane + cell];
        species_moments(md, s, fc[s], &n[s], &jx[s], &jy[s], &E[s]);
      }
      double rho, u, v, t;
      mixture(md, n, jx, jy, E, &rho, &u, &v, &t);
      for (int s = 0; s < S; ++s) {
        double feq[NV];
        or_feq(md, s, n[s], u, v, t, feq);
        for (int k = 0; k < 12; ++k) {
          const double *row = md->M[s] + (k + 4) * NV;
          double acc = 0.0;
          for (int i = 0; i < NV; ++i) acc += (fc[s][i] - feq[i]) * row[i];
          delta[((size_t)s * 12 + k) * plane + cell] = md->sp[s].m * acc;
        }
      }
    }
  }
  if (totals) {
    double mass[OR_MAXS] = {0}, Px = 0, Py = 0, En = 0;
    for (size_t cell = 0; cell < plane; ++cell) {
      for (int s = 0; s < S; ++s) {
        double fc[NV], n, jx, jy, E;
        for (int i = 0; i < NV; ++i) fc[i] = f[((size_t)s * NV + i) * plane + cell];
        species_moments(md, s, fc, &n, &jx, &jy, &E);
        double m = md->sp[s].m;
        mass[s] += m * n;
        Px += m * jx;
        Py += m * jy;
        En += 0.5 * m * E;
      }
    }
    double area = c->dx * c->dy;
    for (int s = 0; s < S; ++s) totals[s] = mass[s] * area;
    totals[S] = Px * area;
    totals[S + 1] = Py * area;
    totals[S + 2] = En * area;
  }
  return 0;
}

/* Energies and energy fluxes of the paragraph after Eqs.(21)-(23): sums over
 * the 16 discrete velocities of m f_i times v_ix^2, v_iy^2, q_i v_ix, q_i v_iy
 * (halved), for f and for f^eq(n^s, u, T) = M^{-1} fhat. */
static void energy_cell(const or_model *md, int s, const double *g, double *out4) {
  double a = 0, b = 0, c = 0, d = 0;
  for (int i = 0; i < NV; ++i) {
    const double vx = md->vx[s][i], vy = md->vy[s][i], q = md->q[s][i];
    a += g[i] * vx * vx;
    b += g[i] * vy * vy;
    c += g[i] * q * vx;
    d += g[i] * q * vy;
  }
  const double hm = 0.5 * md->sp[s].m;
  out4[0] = hm * a; out4[1] = hm * b; out4[2] = hm * c; out4[3] = hm * d;
}

int or_energy(const or_model *md, const double *f, double *fields, double *totals) {
  if (!md || !f) return -1;
  const or_config *c = &md->cfg;
  const int S = c->S;
  const size_t plane = (size_t)c->nx * c->ny;
  if (totals)
    for (int k = 0; k < 8 * S; ++k) totals[k] = 0.0;
  /* cells in order, so that the totals are summed in a fixed order */
  for (size_t cell = 0; cell < plane; ++cell) {
    double fc[OR_MAXS][NV], n[OR_MAXS], jx[OR_MAXS], jy[OR_MAXS], E[OR_MAXS];
    for (int s = 0; s < S; ++s) {
      for (int i = 0; i < NV; ++i) fc[s][i] = f[((size_t)s * NV + i) * plane + cell];
      species_moments(md, s, fc[s], &n[s], &jx[s], &jy[s], &E[s]);
    }
    double rho, u, v, t;
    mixture(md, n, jx, jy, E, &rho, &u, &v, &t);
    for (int s = 0; s < S; ++s) {
      double feq[NV], ef[4], ee[4];
      or_feq(md, s, n[s], u, v, t, feq);
      energy_cell(md, s, fc[s], ef);
      energy_cell(md, s, feq, ee);
      const double vals[8] = {ef[0], ef[1], ee[0], ee[1], ef[2], ef[3], ee[2], ee[3]};
      for (int k = 0; k < 8; ++k) {
        if (fields) fields[((size_t)s * 8 + k) * plane + cell] = vals[k];
        if (totals) totals[s * 8 + k] += vals[k];
      }
    }
  }
  if (totals)
    for (int k = 0; k < 8 * S; ++k) totals[k] *= c->dx * c->dy;
  return 0;
}
