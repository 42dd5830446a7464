/*
 * lagrange_oracle.c -- plain, slow, FP64 CPU oracle of the pure-Lagrangian
 * step ("Lagrangian rezoning" in Table I and Fig. 2a of the ScalSALE paper,
 * arXiv 2209.01983): the mesh moves with the flow and is never remapped.
 *
 * TEST INFRASTRUCTURE. Only the test suite may load this code (it is built
 * into liboracle.so beside sale_oracle.c). It shares no code, header or
 * constant with the HIP path.
 *
 * The paper names the mode and prints no equations. The reading below
 * carries the Eulerian oracle's Lagrangian phase (compatible energy, VNR +
 * Landshoff viscosity, acoustic predictor) over to a deforming hex mesh:
 *
 *   L1  geometry of each cell at t^n from its 8 nodes: the volume V of the
 *       trilinear hex and the corner vectors S_a = dV/dx_a (exact: the
 *       Jacobian determinant is at most quadratic in each reference
 *       coordinate, so 2x2x2 Gauss-Legendre quadrature of det J and of its
 *       derivative is exact); length scale h = V / (largest face area), a
 *       face's area being half the norm of the cross product of its
 *       diagonals;
 *   L2  rho = m/V (cell mass m is constant), p = (gamma-1) rho e,
 *       c = sqrt(gamma (gamma-1) max(e,0)), D = (1/V) sum_a S_a . u_a,
 *       q = rho (C_Q (h D)^2 + C_L c h |D|) where D < 0, else 0;
 *   L3  dt = CFL / max_c (a_c / h_c), a_c = c + max_a |u_a| + 4 C_Q h max(-D,0),
 *       clipped to land on t_end;
 *   L4  predictor: dVs = dt V D / 2, rho_s = m / (V + dVs),
 *       e_s = e - (p+q) dVs / m, P* = (gamma-1) rho_s e_s + q;
 *   L5  viscous hourglass forces (Flanagan & Belytschko, IJNME 17, 1981):
 *       for the four patterns Gamma_k over the corners (sign products
 *       s_y s_z, s_z s_x, s_x s_y, s_x s_y s_z of the corner's reference
 *       octant), gamma_k,a = Gamma_k,a - (1/V) sum_i (sum_b Gamma_k,b x_b^i)
 *       S_a^i (orthogonal to every linear velocity field), g_k = sum_a
 *       gamma_k,a u_a, f_a = -C_HG rho c V^(2/3) sum_k gamma_k,a g_k;
 *   L6  corner forces F_ca = P* S_a + f_a; node force = sum of the corner
 *       forces of its cells; u' = u + dt F / m_p with m_p = 1/8 sum of the
 *       masses of the existing cells around the node; normal components
 *       zeroed on the walls; u_bar = (u + u')/2; x' = x + dt u_bar;
 *   L7  compatible energy: e' = e - (dt/m) sum_a F_ca . u_bar_a;
 *   L8  admissibility: V + dVs > 0, V(x') > 0 (else ETANGLE), e' finite and
 *       >= 0 (else ENUMERIC); nothing is committed on an error.
 *
 * Layout: as the Eulerian oracle (cells x fastest; nodes (nx+1)(ny+1)(nz+1)),
 * node positions x, y, z and velocities u, v, w. Corner a of cell (i,j,k)
 * has bits (a&1, a>>1&1, a>>2&1) and sits at node (i + a&1, j + a>>1&1,
 * k + a>>2&1).
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OLG_OK 0
#define OLG_DONE 1
#define OLG_EINVAL (-1)
#define OLG_ENOMEM (-2)
#define OLG_ENUMERIC (-4)
#define OLG_ETANGLE (-5)

typedef struct {
  int32_t nx, ny, nz;
  double gamma, cfl, cq, cl, chg;
  double t_end;
} olg_config;

static size_t cidx(const olg_config *g, int i, int j, int k) {
  return (size_t)i + (size_t)g->nx * ((size_t)j + (size_t)g->ny * (size_t)k);
}
static size_t nidx(const olg_config *g, int i, int j, int k) {
  return (size_t)i + (size_t)(g->nx + 1) * ((size_t)j + (size_t)(g->ny + 1) * (size_t)k);
}
static int valid(const olg_config *g) {
  return g && g->nx >= 1 && g->ny >= 1 && g->nz >= 1 && g->gamma > 1.0 && g->cfl > 0.0 && g->cq >= 0.0 &&
         g->cl >= 0.0 && g->chg >= 0.0;
}

/* L1: volume and corner vectors of one trilinear hex (X[a][i]: corner a,
 * coordinate i) by 2x2x2 Gauss-Legendre quadrature on the unit cube. */
void olg_hex(const double X[8][3], double S[8][3], double *V) {
  const double gp[2] = {0.5 - 0.5 / sqrt(3.0), 0.5 + 0.5 / sqrt(3.0)};
  double vol = 0.0;
  memset(S, 0, 8 * 3 * sizeof(double));
  for (int q = 0; q < 8; q++) {
    const double r[3] = {gp[q & 1], gp[(q >> 1) & 1], gp[(q >> 2) & 1]};
    double dN[8][3];
    for (int a = 0; a < 8; a++) {
      double L[3], dL[3];
      for (int d = 0; d < 3; d++) {
        const int bit = (a >> d) & 1;
        L[d] = bit ? r[d] : 1.0 - r[d];
        dL[d] = bit ? 1.0 : -1.0;
      }
      dN[a][0] = dL[0] * L[1] * L[2];
      dN[a][1] = L[0] * dL[1] * L[2];
      dN[a][2] = L[0] * L[1] * dL[2];
    }
    double J[3][3] = {{0}};  /* J[d] = dX/dr_d */
    for (int d = 0; d < 3; d++)
      for (int a = 0; a < 8; a++)
        for (int i = 0; i < 3; i++) J[d][i] += dN[a][d] * X[a][i];
    double C[3][3];  /* C[d] = dDet/dJ[d]: cross product of the other two columns */
    for (int d = 0; d < 3; d++) {
      const double *A = J[(d + 1) % 3], *B = J[(d + 2) % 3];
      C[d][0] = A[1] * B[2] - A[2] * B[1];
      C[d][1] = A[2] * B[0] - A[0] * B[2];
      C[d][2] = A[0] * B[1] - A[1] * B[0];
    }
    const double det = J[0][0] * C[0][0] + J[0][1] * C[0][1] + J[0][2] * C[0][2];
    vol += det / 8.0;
    for (int a = 0; a < 8; a++)
      for (int i = 0; i < 3; i++) S[a][i] += (dN[a][0] * C[0][i] + dN[a][1] * C[1][i] + dN[a][2] * C[2][i]) / 8.0;
  }
  *V = vol;
}

/* L1: length scale V / (largest face area) */
double olg_length(const double X[8][3], double V) {
  static const int face[6][4] = {{0, 2, 6, 4}, {1, 3, 7, 5}, {0, 1, 5, 4}, {2, 3, 7, 6}, {0, 1, 3, 2}, {4, 5, 7, 6}};
  double amax = 0.0;
  for (int f = 0; f < 6; f++) {
    double d1[3], d2[3];
    for (int i = 0; i < 3; i++) {
      d1[i] = X[face[f][2]][i] - X[face[f][0]][i];
      d2[i] = X[face[f][3]][i] - X[face[f][1]][i];
    }
    const double cx = d1[1] * d2[2] - d1[2] * d2[1], cy = d1[2] * d2[0] - d1[0] * d2[2],
                 cz = d1[0] * d2[1] - d1[1] * d2[0];
    const double area = 0.5 * sqrt(cx * cx + cy * cy + cz * cz);
    if (area > amax) amax = area;
  }
  return V / amax;
}

static void gather(const olg_config *g, const double *f0, const double *f1, const double *f2, int i, int j, int k,
                   double out[8][3]) {
  for (int a = 0; a < 8; a++) {
    const size_t n = nidx(g, i + (a & 1), j + ((a >> 1) & 1), k + ((a >> 2) & 1));
    out[a][0] = f0[n];
    out[a][1] = f1[n];
    out[a][2] = f2[n];
  }
}

/* L2 + the signal speed of L3 for one cell; returns 0 if V <= 0 */
typedef struct {
  double S[8][3], V, h, rho, p, cs, D, q, a;
} cell_state;

static int cell_eval(const olg_config *g, const double X[8][3], const double U[8][3], double e, double m,
                     cell_state *c) {
  olg_hex(X, c->S, &c->V);
  if (!(c->V > 0.0)) return 0;
  c->h = olg_length(X, c->V);
  c->rho = m / c->V;
  c->p = (g->gamma - 1.0) * c->rho * e;
  c->cs = sqrt(g->gamma * (g->gamma - 1.0) * (e > 0.0 ? e : 0.0));
  double div = 0.0, smax = 0.0;
  for (int a = 0; a < 8; a++) {
    div += c->S[a][0] * U[a][0] + c->S[a][1] * U[a][1] + c->S[a][2] * U[a][2];
    const double s = sqrt(U[a][0] * U[a][0] + U[a][1] * U[a][1] + U[a][2] * U[a][2]);
    if (s > smax) smax = s;
  }
  c->D = div / c->V;
  c->q = 0.0;
  if (c->D < 0.0) {
    const double hd = c->h * c->D;
    c->q = c->rho * (g->cq * hd * hd + g->cl * c->cs * c->h * fabs(c->D));
  }
  c->a = c->cs + smax + 4.0 * g->cq * c->h * (c->D < 0.0 ? -c->D : 0.0);
  return 1;
}

/* L4-L6 for one cell: corner forces F[a] = P* S_a + f_a (hourglass part f).
 * Returns 0 (and zero forces) if V <= 0 or V + dVs <= 0. */
int olg_cell_forces(const olg_config *g, const double X[8][3], const double U[8][3], double e, double m, double dt,
                    double F[8][3]) {
  cell_state c;
  memset(F, 0, 8 * 3 * sizeof(double));
  if (!cell_eval(g, X, U, e, m, &c)) return 0;
  const double dVs = 0.5 * dt * c.V * c.D;
  const double Vs = c.V + dVs;
  if (!(Vs > 0.0)) return 0;
  const double rs = m / Vs;
  const double es = e - (c.p + c.q) * dVs / m;
  const double Ps = (g->gamma - 1.0) * rs * es + c.q;
  double f[8][3] = {{0}};
  const double coef = g->chg * c.rho * c.cs * cbrt(c.V * c.V);
  for (int hk = 0; hk < 4; hk++) {
    double G[8], hx[3] = {0, 0, 0}, gam[8], gk[3] = {0, 0, 0};
    for (int a = 0; a < 8; a++) {
      const double sx = (a & 1) ? 1.0 : -1.0, sy = ((a >> 1) & 1) ? 1.0 : -1.0, sz = ((a >> 2) & 1) ? 1.0 : -1.0;
      G[a] = hk == 0 ? sy * sz : hk == 1 ? sz * sx : hk == 2 ? sx * sy : sx * sy * sz;
      for (int d = 0; d < 3; d++) hx[d] += G[a] * X[a][d];
    }
    for (int a = 0; a < 8; a++) gam[a] = G[a] - (hx[0] * c.S[a][0] + hx[1] * c.S[a][1] + hx[2] * c.S[a][2]) / c.V;
    for (int a = 0; a < 8; a++)
      for (int d = 0; d < 3; d++) gk[d] += gam[a] * U[a][d];
    for (int a = 0; a < 8; a++)
      for (int d = 0; d < 3; d++) f[a][d] -= coef * gam[a] * gk[d];
  }
  for (int a = 0; a < 8; a++)
    for (int d = 0; d < 3; d++) F[a][d] = Ps * c.S[a][d] + f[a][d];
  return 1;
}

/* L3: the time step of the current state. OLG_DONE (dt = 0) once t >= t_end. */
int olg_timestep(const olg_config *g, const double *x, const double *y, const double *z, const double *u,
                 const double *v, const double *w, const double *e, const double *m, double t, double *dt) {
  if (!valid(g)) return OLG_EINVAL;
  *dt = 0.0;
  if (t >= g->t_end) return OLG_DONE;
  double rmax = 0.0;
  int bad = 0;
  for (int k = 0; k < g->nz; k++)
    for (int j = 0; j < g->ny; j++)
      for (int i = 0; i < g->nx; i++) {
        double X[8][3], U[8][3];
        gather(g, x, y, z, i, j, k, X);
        gather(g, u, v, w, i, j, k, U);
        cell_state c;
        const size_t ci = cidx(g, i, j, k);
        if (!cell_eval(g, X, U, e[ci], m[ci], &c)) {
          bad = 1;
          continue;
        }
        const double r = c.a / c.h;
        if (!(r <= rmax)) rmax = r;  /* NaN propagates */
      }
  if (bad) return OLG_ETANGLE;
  const double rem = g->t_end - t;
  double d = rmax > 0.0 ? g->cfl / rmax : rem;
  if (d > rem) d = rem;
  if (!(d > 0.0) || !isfinite(d)) return OLG_ENUMERIC;
  *dt = d;
  return OLG_OK;
}

/* One whole step (L1..L8) in place; *dt_used = the step's dt. */
int olg_step(const olg_config *g, double *x, double *y, double *z, double *u, double *v, double *w, double *e,
             const double *m, double *t, double *dt_used) {
  double dt;
  int rc = olg_timestep(g, x, y, z, u, v, w, e, m, *t, &dt);
  if (dt_used) *dt_used = dt;
  if (rc != OLG_OK) return rc;
  const int nx = g->nx, ny = g->ny, nz = g->nz;
  const size_t nc = (size_t)nx * ny * nz, nn = (size_t)(nx + 1) * (ny + 1) * (nz + 1);
  double *F = malloc(nc * 24 * sizeof(double));  /* corner forces F[c][a][i] */
  double *nu = malloc(nn * 3 * sizeof(double));  /* u' */
  double *ub = malloc(nn * 3 * sizeof(double));  /* u_bar */
  double *en = malloc(nc * sizeof(double));
  if (!F || !nu || !ub || !en) {
    free(F), free(nu), free(ub), free(en);
    return OLG_ENOMEM;
  }
  int tangle = 0, numeric = 0;
  /* L1, L2, L4, L5, L6 (corner forces) */
#pragma omp parallel for collapse(2) schedule(static) reduction(| : tangle)
  for (int k = 0; k < nz; k++)
    for (int j = 0; j < ny; j++)
      for (int i = 0; i < nx; i++) {
        const size_t ci = cidx(g, i, j, k);
        double X[8][3], U[8][3];
        gather(g, x, y, z, i, j, k, X);
        gather(g, u, v, w, i, j, k, U);
        double *Fc = F + 24 * ci;
        if (!olg_cell_forces(g, X, U, e[ci], m[ci], dt, (double(*)[3])Fc)) tangle = 1;
      }
  /* L6: node forces, u', u_bar, x' */
#pragma omp parallel for collapse(2) schedule(static)
  for (int k = 0; k <= nz; k++)
    for (int j = 0; j <= ny; j++)
      for (int i = 0; i <= nx; i++) {
        double Fn[3] = {0, 0, 0}, mp = 0.0;
        for (int a = 0; a < 8; a++) {  /* the node is corner a of cell (i,j,k) - bits(a) */
          const int ci = i - (a & 1), cj = j - ((a >> 1) & 1), ck = k - ((a >> 2) & 1);
          if (ci < 0 || ci >= nx || cj < 0 || cj >= ny || ck < 0 || ck >= nz) continue;
          const size_t c = cidx(g, ci, cj, ck);
          for (int d = 0; d < 3; d++) Fn[d] += F[24 * c + 3 * a + d];
          mp += m[c];
        }
        mp *= 0.125;
        const size_t n = nidx(g, i, j, k);
        const double uo[3] = {u[n], v[n], w[n]};
        double un[3];
        for (int d = 0; d < 3; d++) un[d] = uo[d] + dt * Fn[d] / mp;
        if (i == 0 || i == nx) un[0] = 0.0;
        if (j == 0 || j == ny) un[1] = 0.0;
        if (k == 0 || k == nz) un[2] = 0.0;
        for (int d = 0; d < 3; d++) {
          nu[3 * n + d] = un[d];
          ub[3 * n + d] = 0.5 * (uo[d] + un[d]);
        }
      }
  /* L7 */
#pragma omp parallel for collapse(2) schedule(static) reduction(| : numeric)
  for (int k = 0; k < nz; k++)
    for (int j = 0; j < ny; j++)
      for (int i = 0; i < nx; i++) {
        const size_t ci = cidx(g, i, j, k);
        double work = 0.0;
        for (int a = 0; a < 8; a++) {
          const size_t n = nidx(g, i + (a & 1), j + ((a >> 1) & 1), k + ((a >> 2) & 1));
          for (int d = 0; d < 3; d++) work += F[24 * ci + 3 * a + d] * ub[3 * n + d];
        }
        en[ci] = e[ci] - dt * work / m[ci];
        if (!isfinite(en[ci]) || !(en[ci] >= 0.0)) numeric = 1;
      }
  /* L8: new positions must give positive volumes */
  double *xn = malloc(nn * 3 * sizeof(double));
  if (!xn) {
    free(F), free(nu), free(ub), free(en);
    return OLG_ENOMEM;
  }
  for (size_t n = 0; n < nn; n++) {
    xn[3 * n + 0] = x[n] + dt * ub[3 * n + 0];
    xn[3 * n + 1] = y[n] + dt * ub[3 * n + 1];
    xn[3 * n + 2] = z[n] + dt * ub[3 * n + 2];
  }
#pragma omp parallel for collapse(2) schedule(static) reduction(| : tangle)
  for (int k = 0; k < nz; k++)
    for (int j = 0; j < ny; j++)
      for (int i = 0; i < nx; i++) {
        double X[8][3], S[8][3], V;
        for (int a = 0; a < 8; a++) {
          const size_t n = nidx(g, i + (a & 1), j + ((a >> 1) & 1), k + ((a >> 2) & 1));
          for (int d = 0; d < 3; d++) X[a][d] = xn[3 * n + d];
        }
        olg_hex(X, S, &V);
        if (!(V > 0.0)) tangle = 1;
      }
  if (!tangle && !numeric) {
    for (size_t n = 0; n < nn; n++) {
      x[n] = xn[3 * n + 0], y[n] = xn[3 * n + 1], z[n] = xn[3 * n + 2];
      u[n] = nu[3 * n + 0], v[n] = nu[3 * n + 1], w[n] = nu[3 * n + 2];
    }
    memcpy(e, en, nc * sizeof(double));
    *t = *t + dt;
  }
  free(F), free(nu), free(ub), free(en), free(xn);
  if (tangle) return OLG_ETANGLE;
  if (numeric) return OLG_ENUMERIC;
  return OLG_OK;
}

/* density of every cell, m / V(x) */
int olg_density(const olg_config *g, const double *x, const double *y, const double *z, const double *m,
                double *rho) {
  if (!valid(g)) return OLG_EINVAL;
  for (int k = 0; k < g->nz; k++)
    for (int j = 0; j < g->ny; j++)
      for (int i = 0; i < g->nx; i++) {
        double X[8][3], S[8][3], V;
        gather(g, x, y, z, i, j, k, X);
        olg_hex(X, S, &V);
        rho[cidx(g, i, j, k)] = m[cidx(g, i, j, k)] / V;
      }
  return OLG_OK;
}
