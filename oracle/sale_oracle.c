/*
 * sale_oracle.c -- plain, slow, FP64 CPU oracle for one SALE step
 * (staggered Lagrangian phase followed by an Eulerian donor-cell remap back
 * to the fixed mesh) on a logically structured 3D hex mesh.
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library. It shares no code,
 * header or constant with the HIP path.
 *
 * What the ScalSALE paper fixes (arXiv 2209.01983):
 *   - a SALE hydro scheme with a Lagrangian kernel, an Eulerian rezone and an
 *     advection phase on a structured grid (Sec. I-D, Table I);
 *   - the ideal-gas equation of state (Sec. I-C/I-D);
 *   - vertex quantities beside cell quantities (Sec. III-C/III-D);
 *   - density computed in the hydro module (Sec. III-A);
 *   - Sod and Sedov-Taylor as verification flows (Sec. I-D, Fig. 2).
 * The paper prints no equations for the scheme. Every formula below is the
 * oracle's own fixed reading, from standard staggered-grid practice:
 * compatible total-energy differencing (Caramana, Burton, Shashkov & Whalen,
 * J. Comput. Phys. 146, 1998), a von Neumann-Richtmyer quadratic plus
 * Landshoff linear artificial viscosity, an acoustic half-step pressure
 * predictor, exact trilinear swept volumes, a first-order unsplit donor-cell
 * face-flux remap, a dual-mesh momentum remap and a DeBar-style kinetic
 * energy fix. The step labels O1..O12 below name those readings.
 *
 * Layout: cell (i,j,k) -> i + nx*(j + ny*k); node (i,j,k), 0<=i<=nx ->
 * i + (nx+1)*(j + (ny+1)*k). Velocity is three node arrays u, v, w.
 * All six faces are reflective walls.
 *
 * Parallelism: OpenMP "parallel for" over independent cells or nodes only;
 * every output element is written by one thread in a fixed order, so the
 * results do not depend on the thread count. Reductions (max, sums) are
 * serial.
 */
#define _GNU_SOURCE
#include <math.h>
#include <omp.h>
#include <sys/mman.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_DONE 1
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_ENUMERIC (-4)
#define ORC_ETANGLE (-5)

typedef struct {
  int32_t nx, ny, nz;
  double lo[3], hi[3];
  double gamma, cfl, cq, cl;
  double t_end;
  int32_t order; /* remap order: 1 (donor cell) or 2 (limited linear) */
} orc_config;

/* Scratch arrays of one step. Face arrays: x faces (nx+1)*ny*nz,
 * y faces nx*(ny+1)*nz, z faces nx*ny*(nz+1). */
typedef struct {
  int32_t nx, ny, nz;
  double *p, *c, *q, *D, *ps, *mc;          /* cells */
  double *mp, *u1, *v1, *w1, *ub, *vb, *wb; /* nodes */
  double *eL, *VL, *rhoL;                   /* cells */
  double *dvx, *dvy, *dvz;                  /* faces: swept volumes */
  double *mux, *muy, *muz;                  /* faces: mass fluxes */
  double *ex, *ey, *ez;                     /* faces: internal-energy fluxes */
  double *M, *E, *epre, *rn;                /* cells; rn = new density */
  double *P1, *P2, *P3, *K, *mn, *dK;       /* nodes */
  double *un, *vn, *wn;                     /* nodes: new velocity */
  double *sr[3], *se[3];                    /* cells: limited slopes of rho^L, e^L */
} orc_ws;

/* ------------------------------------------------------------------ */
/* index helpers                                                        */
/* ------------------------------------------------------------------ */
#define NX (g->nx)
#define NY (g->ny)
#define NZ (g->nz)
static inline size_t CI(const orc_config *g, int i, int j, int k) {
  return (size_t)i + (size_t)NX * ((size_t)j + (size_t)NY * (size_t)k);
}
static inline size_t NI(const orc_config *g, int i, int j, int k) {
  return (size_t)i + (size_t)(NX + 1) * ((size_t)j + (size_t)(NY + 1) * (size_t)k);
}
static inline size_t FXI(const orc_config *g, int i, int j, int k) {
  return (size_t)i + (size_t)(NX + 1) * ((size_t)j + (size_t)NY * (size_t)k);
}
static inline size_t FYI(const orc_config *g, int i, int j, int k) {
  return (size_t)i + (size_t)NX * ((size_t)j + (size_t)(NY + 1) * (size_t)k);
}
static inline size_t FZI(const orc_config *g, int i, int j, int k) {
  return (size_t)i + (size_t)NX * ((size_t)j + (size_t)NY * (size_t)k);
}
static inline int cell_exists(const orc_config *g, int i, int j, int k) {
  return i >= 0 && i < NX && j >= 0 && j < NY && k >= 0 && k < NZ;
}
static inline int node_exists(const orc_config *g, int i, int j, int k) {
  return i >= 0 && i <= NX && j >= 0 && j <= NY && k >= 0 && k <= NZ;
}

static void spacing(const orc_config *g, double *dx, double *dy, double *dz) {
  *dx = (g->hi[0] - g->lo[0]) / (double)NX;
  *dy = (g->hi[1] - g->lo[1]) / (double)NY;
  *dz = (g->hi[2] - g->lo[2]) / (double)NZ;
}

/* Corner vectors of a Cartesian cell: S_{c,p} = dV_c/dx_p for the corner p at
 * octant signs (sx,sy,sz) in {-1,+1}^3 relative to the cell centre is
 * (sx*dy*dz, sy*dz*dx, sz*dx*dy)/4. Every sum over the eight corners of a
 * cell, sum_p S_{c,p}.X_p, is evaluated here grouped as differences across
 * the cell along each axis (the +side corner minus the -side corner of the
 * same edge), a reordering that makes a uniform X give exactly zero. */
static double corner_sum(const orc_config *g, double dx, double dy, double dz, int i, int j,
                         int k, const double *X, const double *Y, const double *Z) {
  double sx = 0.0, sy = 0.0, sz = 0.0;
  for (int t2 = 0; t2 < 2; t2++)
    for (int t1 = 0; t1 < 2; t1++) {
      sx += X[NI(g, i + 1, j + t1, k + t2)] - X[NI(g, i, j + t1, k + t2)];
      sy += Y[NI(g, i + t1, j + 1, k + t2)] - Y[NI(g, i + t1, j, k + t2)];
      sz += Z[NI(g, i + t1, j + t2, k + 1)] - Z[NI(g, i + t1, j + t2, k)];
    }
  return (dy * dz / 4.0) * sx + (dz * dx / 4.0) * sy + (dx * dy / 4.0) * sz;
}

/* ------------------------------------------------------------------ */
/* workspace                                                            */
/* ------------------------------------------------------------------ */
void orc_ws_destroy(orc_ws *w);

/* malloc + zero-fill in parallel (first touch spread over the threads, so
 * that the page faults of a multi-GB workspace do not serialise). */
static double *zalloc(size_t n) {
  void *v = NULL;
  size_t bytes = n * sizeof(double) + 64;
  if (posix_memalign(&v, (size_t)1 << 21, bytes) != 0) return NULL;
  madvise(v, bytes, MADV_HUGEPAGE); /* fewer page faults on GB-sized arrays */
  double *p = (double *)v;
#pragma omp parallel for schedule(static)
  for (size_t a = 0; a < n; a++) p[a] = 0.0;
  return p;
}

orc_ws *orc_ws_create(const orc_config *g) {
  if (!g || g->nx < 1 || g->ny < 1 || g->nz < 1) return NULL;
  orc_ws *w = (orc_ws *)calloc(1, sizeof(orc_ws));
  if (!w) return NULL;
  w->nx = g->nx; w->ny = g->ny; w->nz = g->nz;
  size_t nc = (size_t)NX * NY * NZ;
  size_t nn = (size_t)(NX + 1) * (NY + 1) * (NZ + 1);
  size_t nfx = (size_t)(NX + 1) * NY * NZ, nfy = (size_t)NX * (NY + 1) * NZ,
         nfz = (size_t)NX * NY * (NZ + 1);
  double **cells[] = {&w->p,  &w->c,  &w->q,     &w->D,     &w->ps,    &w->mc,    &w->eL,
                      &w->VL, &w->rhoL, &w->M, &w->E,  &w->epre,  &w->rn,    &w->sr[0],
                      &w->sr[1], &w->sr[2], &w->se[0], &w->se[1], &w->se[2]};
  double **nodes[] = {&w->mp, &w->u1, &w->v1, &w->w1, &w->ub, &w->vb, &w->wb, &w->P1,
                      &w->P2, &w->P3, &w->K, &w->mn, &w->dK, &w->un, &w->vn, &w->wn};
  int ok = 1;
  for (size_t a = 0; a < sizeof(cells) / sizeof(cells[0]); a++)
    ok &= (*cells[a] = zalloc(nc)) != NULL;
  for (size_t a = 0; a < sizeof(nodes) / sizeof(nodes[0]); a++)
    ok &= (*nodes[a] = zalloc(nn)) != NULL;
  ok &= (w->dvx = zalloc(nfx)) != NULL;
  ok &= (w->mux = zalloc(nfx)) != NULL;
  ok &= (w->ex = zalloc(nfx)) != NULL;
  ok &= (w->dvy = zalloc(nfy)) != NULL;
  ok &= (w->muy = zalloc(nfy)) != NULL;
  ok &= (w->ey = zalloc(nfy)) != NULL;
  ok &= (w->dvz = zalloc(nfz)) != NULL;
  ok &= (w->muz = zalloc(nfz)) != NULL;
  ok &= (w->ez = zalloc(nfz)) != NULL;
  if (!ok) { orc_ws_destroy(w); return NULL; }
  return w;
}

void orc_ws_destroy(orc_ws *w) {
  if (!w) return;
  double *all[] = {w->p, w->c, w->q, w->D, w->ps, w->mc, w->mp, w->u1, w->v1, w->w1,
                   w->ub, w->vb, w->wb, w->eL, w->VL, w->rhoL, w->dvx, w->dvy, w->dvz,
                   w->mux, w->muy, w->muz, w->ex, w->ey, w->ez, w->M, w->E, w->epre, w->rn,
                   w->P1, w->P2, w->P3, w->K, w->mn, w->dK, w->un, w->vn, w->wn,
                   w->sr[0], w->sr[1], w->sr[2], w->se[0], w->se[1], w->se[2]};
  for (size_t a = 0; a < sizeof(all) / sizeof(all[0]); a++) free(all[a]);
  free(w);
}

static int config_valid(const orc_config *g) {
  if (!g || g->nx < 1 || g->ny < 1 || g->nz < 1) return 0;
  for (int a = 0; a < 3; a++)
    if (!(g->hi[a] > g->lo[a])) return 0;
  if (!(g->gamma > 1.0) || !(g->cfl > 0.0) || !(g->cfl < 1.0)) return 0;
  if (!(g->cq >= 0.0) || !(g->cl >= 0.0) || !(g->t_end >= 0.0)) return 0;
  if (g->order != 1 && g->order != 2) return 0;
  return 1;
}

/* ------------------------------------------------------------------ */
/* O8 kernel: swept volume of one face                                  */
/* ------------------------------------------------------------------ */
/* Exact volume swept when a planar rectangular face (edge lengths h1 along
 * its first tangent, h2 along its second; tangents cyclic after the normal)
 * moves by a displacement field bilinear in the face parameters (s,t).
 * d[q][m]: displacement at corner q in the order (s,t) = (0,0), (1,0), (0,1),
 * (1,1); component m = 0 along the normal, 1 along tangent 1, 2 along
 * tangent 2. The volume is the integral over r, s, t in [0,1] of the
 * Jacobian of X(s,t) + r*delta(s,t); after the r integration the integrand
 * in (s,t) has degree <= 2 in each variable, so the 2x2 Gauss-Legendre rule
 * below is exact. Positive when the face moves toward +normal. */
double orc_face_swept_volume(const double d[4][3], double h1, double h2) {
  const double gp[2] = {0.5 - 0.5 / sqrt(3.0), 0.5 + 0.5 / sqrt(3.0)};
  double vol = 0.0;
  for (int a = 0; a < 2; a++) {
    for (int b = 0; b < 2; b++) {
      double s = gp[a], t = gp[b];
      double del[3], ds[3], dt[3];
      for (int m = 0; m < 3; m++) {
        del[m] = d[0][m] * (1 - s) * (1 - t) + d[1][m] * s * (1 - t) +
                 d[2][m] * (1 - s) * t + d[3][m] * s * t;
        ds[m] = (d[1][m] - d[0][m]) * (1 - t) + (d[3][m] - d[2][m]) * t;
        dt[m] = (d[2][m] - d[0][m]) * (1 - s) + (d[3][m] - d[1][m]) * s;
      }
      double xi = del[0], eta = del[1], zeta = del[2];
      double cr[3] = {ds[1] * dt[2] - ds[2] * dt[1], ds[2] * dt[0] - ds[0] * dt[2],
                      ds[0] * dt[1] - ds[1] * dt[0]};
      double triple = del[0] * cr[0] + del[1] * cr[1] + del[2] * cr[2];
      double f = h1 * h2 * xi + 0.5 * h1 * (xi * dt[2] - zeta * dt[0]) +
                 0.5 * h2 * (xi * ds[1] - eta * ds[0]) + triple / 3.0;
      vol += 0.25 * f;
    }
  }
  return vol;
}

/* ------------------------------------------------------------------ */
/* O1, O2, O4, O3: masses, EOS, divergence, viscosity, time step        */
/* ------------------------------------------------------------------ */
static void stage_cells_eos_div_q(const orc_config *g, const double *rho, const double *e,
                                  const double *u, const double *v, const double *w,
                                  orc_ws *W) {
  double dx, dy, dz;
  spacing(g, &dx, &dy, &dz);
  const double V0 = dx * dy * dz, h = fmin(dx, fmin(dy, dz)), gm = g->gamma;
#pragma omp parallel for schedule(static)
  for (int k = 0; k < NZ; k++)
    for (int j = 0; j < NY; j++)
      for (int i = 0; i < NX; i++) {
        size_t c = CI(g, i, j, k);
        W->mc[c] = rho[c] * V0;                               /* O1 */
        W->p[c] = (gm - 1.0) * rho[c] * e[c];                 /* O2 */
        W->c[c] = sqrt(gm * (gm - 1.0) * fmax(e[c], 0.0));
        double div = corner_sum(g, dx, dy, dz, i, j, k, u, v, w); /* O4 */
        W->D[c] = div / V0;
        if (W->D[c] < 0.0) {
          double hd = h * W->D[c];
          W->q[c] = rho[c] * (g->cq * hd * hd + g->cl * W->c[c] * h * fabs(W->D[c]));
        } else {
          W->q[c] = 0.0;
        }
      }
}

static void stage_nodal_mass(const orc_config *g, const double *mc, double *mp) {
#pragma omp parallel for schedule(static)
  for (int k = 0; k <= NZ; k++)
    for (int j = 0; j <= NY; j++)
      for (int i = 0; i <= NX; i++) {
        double s = 0.0;
        for (int cc = -1; cc <= 0; cc++)
          for (int b = -1; b <= 0; b++)
            for (int a = -1; a <= 0; a++)
              if (cell_exists(g, i + a, j + b, k + cc)) s += mc[CI(g, i + a, j + b, k + cc)];
        mp[NI(g, i, j, k)] = 0.125 * s;
      }
}

/* O3 precondition: the state is admissible (rho > 0, e >= 0, all finite). */
static int state_admissible(const orc_config *g, const double *rho, const double *e,
                            const double *u, const double *v, const double *w) {
  size_t nc = (size_t)NX * NY * NZ, nn = (size_t)(NX + 1) * (NY + 1) * (NZ + 1);
  for (size_t c = 0; c < nc; c++)
    if (!(rho[c] > 0.0) || !isfinite(rho[c]) || !(e[c] >= 0.0) || !isfinite(e[c])) return 0;
  for (size_t n = 0; n < nn; n++)
    if (!isfinite(u[n]) || !isfinite(v[n]) || !isfinite(w[n])) return 0;
  return 1;
}

/* O3: largest signal speed of the current state over all cells. */
static double stage_max_signal(const orc_config *g, const double *u, const double *v,
                               const double *w, const orc_ws *W) {
  double dx, dy, dz;
  spacing(g, &dx, &dy, &dz);
  const double h = fmin(dx, fmin(dy, dz));
  double amax = 0.0;
  for (int k = 0; k < NZ; k++)
    for (int j = 0; j < NY; j++)
      for (int i = 0; i < NX; i++) {
        size_t c = CI(g, i, j, k);
        double s = 0.0;
        for (int cc = 0; cc < 2; cc++)
          for (int b = 0; b < 2; b++)
            for (int a = 0; a < 2; a++) {
              size_t n = NI(g, i + a, j + b, k + cc);
              double sp = sqrt(u[n] * u[n] + v[n] * v[n] + w[n] * w[n]);
              if (sp > s) s = sp;
            }
        double ac = W->c[c] + s + 4.0 * g->cq * h * fmax(-W->D[c], 0.0);
        if (isnan(ac) || isnan(amax)) amax = NAN; /* a NaN anywhere poisons dt */
        else if (ac > amax) amax = ac;
      }
  return amax;
}

/* ------------------------------------------------------------------ */
/* O5: acoustic predictor                                               */
/* ------------------------------------------------------------------ */
static int stage_predictor(const orc_config *g, const double *rho, const double *e, double dt,
                           orc_ws *W) {
  double dx, dy, dz;
  spacing(g, &dx, &dy, &dz);
  const double V0 = dx * dy * dz, gm = g->gamma;
  size_t nc = (size_t)NX * NY * NZ;
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (size_t c = 0; c < nc; c++) {
    double dVs = 0.5 * dt * V0 * W->D[c];
    double Vs = V0 + dVs;
    if (!(Vs > 0.0)) { bad |= 1; W->ps[c] = 0.0; continue; }
    double rs = W->mc[c] / Vs;
    double es = e[c] - (W->p[c] + W->q[c]) * dVs / W->mc[c];
    W->ps[c] = (gm - 1.0) * rs * es + W->q[c];
    (void)rho;
  }
  return bad ? ORC_ETANGLE : ORC_OK;
}

/* ------------------------------------------------------------------ */
/* O6: forces, velocity, walls, mean velocity                           */
/* ------------------------------------------------------------------ */
static double ps_at(const orc_config *g, const orc_ws *W, int i, int j, int k) {
  return cell_exists(g, i, j, k) ? W->ps[CI(g, i, j, k)] : 0.0;
}

static void stage_forces_motion(const orc_config *g, const double *u, const double *v,
                                const double *w, double dt, orc_ws *W) {
  double dx, dy, dz;
  spacing(g, &dx, &dy, &dz);
#pragma omp parallel for schedule(static)
  for (int k = 0; k <= NZ; k++)
    for (int j = 0; j <= NY; j++)
      for (int i = 0; i <= NX; i++) {
        size_t n = NI(g, i, j, k);
        /* F_p = sum over the existing cells c around p of P*_c S_{c,p}:
         * the node is the +x corner of the cells at i-1 and the -x corner of
         * those at i, so per axis it is (area/4) * sum over the four cell
         * pairs of (P*_lower - P*_upper); a missing cell contributes zero. */
        double F[3] = {0.0, 0.0, 0.0};
        for (int t2 = 0; t2 < 2; t2++)
          for (int t1 = 0; t1 < 2; t1++) {
            F[0] += ps_at(g, W, i - 1, j - t1, k - t2) - ps_at(g, W, i, j - t1, k - t2);
            F[1] += ps_at(g, W, i - t1, j - 1, k - t2) - ps_at(g, W, i - t1, j, k - t2);
            F[2] += ps_at(g, W, i - t1, j - t2, k - 1) - ps_at(g, W, i - t1, j - t2, k);
          }
        F[0] *= dy * dz / 4.0;
        F[1] *= dz * dx / 4.0;
        F[2] *= dx * dy / 4.0;
        double m = W->mp[n];
        double u1 = u[n] + dt * F[0] / m;
        double v1 = v[n] + dt * F[1] / m;
        double w1 = w[n] + dt * F[2] / m;
        if (i == 0 || i == NX) u1 = 0.0;
        if (j == 0 || j == NY) v1 = 0.0;
        if (k == 0 || k == NZ) w1 = 0.0;
        W->u1[n] = u1; W->v1[n] = v1; W->w1[n] = w1;
        W->ub[n] = 0.5 * (u[n] + u1);
        W->vb[n] = 0.5 * (v[n] + v1);
        W->wb[n] = 0.5 * (w[n] + w1);
      }
}

/* ------------------------------------------------------------------ */
/* O7: compatible internal energy                                       */
/* ------------------------------------------------------------------ */
static void stage_compatible_energy(const orc_config *g, const double *e, double dt, orc_ws *W) {
  double dx, dy, dz;
  spacing(g, &dx, &dy, &dz);
#pragma omp parallel for schedule(static)
  for (int k = 0; k < NZ; k++)
    for (int j = 0; j < NY; j++)
      for (int i = 0; i < NX; i++) {
        size_t c = CI(g, i, j, k);
        double work = corner_sum(g, dx, dy, dz, i, j, k, W->ub, W->vb, W->wb);
        W->eL[c] = e[c] - (dt / W->mc[c]) * W->ps[c] * work;
      }
}

/* ------------------------------------------------------------------ */
/* O8: swept volumes of interior faces, Lagrangian volume and density   */
/* ------------------------------------------------------------------ */
static void node_disp(const orc_ws *W, size_t n, double dt, double out[3]) {
  out[0] = dt * W->ub[n];
  out[1] = dt * W->vb[n];
  out[2] = dt * W->wb[n];
}

static int stage_geometry(const orc_config *g, double dt, orc_ws *W) {
  double dx, dy, dz;
  spacing(g, &dx, &dy, &dz);
  const double V0 = dx * dy * dz;
  /* x faces: node plane i, tangents (y, z); corner (s,t)=(b,c) -> node (i, j+b, k+c) */
#pragma omp parallel for schedule(static)
  for (int k = 0; k < NZ; k++)
    for (int j = 0; j < NY; j++)
      for (int i = 0; i <= NX; i++) {
        double vol = 0.0;
        if (i > 0 && i < NX) {
          double d[4][3];
          for (int q = 0; q < 4; q++) {
            int sb = q & 1, tc = q >> 1;
            double dd[3];
            node_disp(W, NI(g, i, j + sb, k + tc), dt, dd);
            d[q][0] = dd[0]; d[q][1] = dd[1]; d[q][2] = dd[2];
          }
          vol = orc_face_swept_volume((const double(*)[3])d, dy, dz);
        }
        W->dvx[FXI(g, i, j, k)] = vol;
      }
  /* y faces: node plane j, tangents (z, x); corner (s,t) -> node (i+t, j, k+s) */
#pragma omp parallel for schedule(static)
  for (int k = 0; k < NZ; k++)
    for (int j = 0; j <= NY; j++)
      for (int i = 0; i < NX; i++) {
        double vol = 0.0;
        if (j > 0 && j < NY) {
          double d[4][3];
          for (int q = 0; q < 4; q++) {
            int s = q & 1, t = q >> 1;
            double dd[3];
            node_disp(W, NI(g, i + t, j, k + s), dt, dd);
            d[q][0] = dd[1]; d[q][1] = dd[2]; d[q][2] = dd[0];
          }
          vol = orc_face_swept_volume((const double(*)[3])d, dz, dx);
        }
        W->dvy[FYI(g, i, j, k)] = vol;
      }
  /* z faces: node plane k, tangents (x, y); corner (s,t) -> node (i+s, j+t, k) */
#pragma omp parallel for schedule(static)
  for (int k = 0; k <= NZ; k++)
    for (int j = 0; j < NY; j++)
      for (int i = 0; i < NX; i++) {
        double vol = 0.0;
        if (k > 0 && k < NZ) {
          double d[4][3];
          for (int q = 0; q < 4; q++) {
            int s = q & 1, t = q >> 1;
            double dd[3];
            node_disp(W, NI(g, i + s, j + t, k), dt, dd);
            d[q][0] = dd[2]; d[q][1] = dd[0]; d[q][2] = dd[1];
          }
          vol = orc_face_swept_volume((const double(*)[3])d, dx, dy);
        }
        W->dvz[FZI(g, i, j, k)] = vol;
      }
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int k = 0; k < NZ; k++)
    for (int j = 0; j < NY; j++)
      for (int i = 0; i < NX; i++) {
        size_t c = CI(g, i, j, k);
        double dV = (W->dvx[FXI(g, i + 1, j, k)] - W->dvx[FXI(g, i, j, k)]) +
                    (W->dvy[FYI(g, i, j + 1, k)] - W->dvy[FYI(g, i, j, k)]) +
                    (W->dvz[FZI(g, i, j, k + 1)] - W->dvz[FZI(g, i, j, k)]);
        W->VL[c] = V0 + dV;
        if (!(W->VL[c] > 0.0)) { bad |= 1; W->rhoL[c] = 0.0; continue; }
        W->rhoL[c] = W->mc[c] / W->VL[c];
      }
  return bad ? ORC_ETANGLE : ORC_OK;
}

/* ------------------------------------------------------------------ */
/* O9: first-order donor-cell face fluxes and cell remap                */
/* ------------------------------------------------------------------ */
/* flux through an interior face between cell L (lower) and R (upper) */
static void donor_flux(const orc_ws *W, double dv, size_t L, size_t R, double *mu, double *eps) {
  size_t dn = (dv > 0.0) ? L : R;
  *mu = W->rhoL[dn] * dv;
  *eps = *mu * W->eL[dn];
}

/* Second-order remap (order 2): the donor's value is taken from a limited
 * linear reconstruction along the face normal, at the centroid of the swept
 * volume. The harmonic (van Leer) limiter of the one-sided differences
 * a_minus, a_plus (per unit length): zero unless they share a sign. */
double orc_vanleer(double a_minus, double a_plus) {
  return (a_minus * a_plus > 0.0) ? 2.0 * a_minus * a_plus / (a_minus + a_plus) : 0.0;
}

/* Donor value at the swept volume's centroid: the donor's value q plus its
 * slope times the signed distance from its centre. The swept slab of
 * thickness |dvA| (= |swept volume| / face area) lies at the donor's end
 * next to the face, so its centroid is (h - |dvA|) / 2 from the donor's
 * centre: toward +axis when the donor is the lower cell (dvA > 0), toward
 * -axis when it is the upper one. */
double orc_donor_value(double q, double slope, double h, double dvA) {
  const double off = 0.5 * (h - fabs(dvA));
  return (dvA > 0.0) ? q + slope * off : q - slope * off;
}

/* limited slopes of rho^L and e^L in every cell along each axis (zero in a
 * cell whose neighbour along that axis is a wall) */
static void stage_cell_slopes(const orc_config *g, orc_ws *W) {
  double hs[3];
  spacing(g, &hs[0], &hs[1], &hs[2]);
#pragma omp parallel for schedule(static)
  for (int k = 0; k < NZ; k++)
    for (int j = 0; j < NY; j++)
      for (int i = 0; i < NX; i++) {
        const size_t c = CI(g, i, j, k);
        for (int a = 0; a < 3; a++) {
          const int di = a == 0, dj = a == 1, dk = a == 2;
          double sr = 0.0, se = 0.0;
          if (cell_exists(g, i - di, j - dj, k - dk) && cell_exists(g, i + di, j + dj, k + dk)) {
            const size_t cm = CI(g, i - di, j - dj, k - dk), cp = CI(g, i + di, j + dj, k + dk);
            sr = orc_vanleer((W->rhoL[c] - W->rhoL[cm]) / hs[a], (W->rhoL[cp] - W->rhoL[c]) / hs[a]);
            se = orc_vanleer((W->eL[c] - W->eL[cm]) / hs[a], (W->eL[cp] - W->eL[c]) / hs[a]);
          }
          W->sr[a][c] = sr;
          W->se[a][c] = se;
        }
      }
}

/* second-order flux through an interior face normal to `axis` */
static void donor_flux2(const orc_ws *W, int axis, double h, double area, double dv, size_t L, size_t R,
                        double *mu, double *eps) {
  const size_t dn = (dv > 0.0) ? L : R;
  const double dvA = dv / area;
  const double rf = orc_donor_value(W->rhoL[dn], W->sr[axis][dn], h, dvA);
  const double ef = orc_donor_value(W->eL[dn], W->se[axis][dn], h, dvA);
  *mu = rf * dv;
  *eps = *mu * ef;
}

static int stage_cell_remap(const orc_config *g, const double *rho, orc_ws *W) {
  double dx, dy, dz;
  spacing(g, &dx, &dy, &dz);
  const double V0 = dx * dy * dz;
  const int o2 = g->order == 2;
  if (o2) stage_cell_slopes(g, W);
#pragma omp parallel for schedule(static)
  for (int k = 0; k < NZ; k++)
    for (int j = 0; j < NY; j++)
      for (int i = 0; i <= NX; i++) {
        size_t f = FXI(g, i, j, k);
        double mu = 0.0, eps = 0.0;
        if (i > 0 && i < NX) {
          if (o2)
            donor_flux2(W, 0, dx, dy * dz, W->dvx[f], CI(g, i - 1, j, k), CI(g, i, j, k), &mu, &eps);
          else
            donor_flux(W, W->dvx[f], CI(g, i - 1, j, k), CI(g, i, j, k), &mu, &eps);
        }
        W->mux[f] = mu; W->ex[f] = eps;
      }
#pragma omp parallel for schedule(static)
  for (int k = 0; k < NZ; k++)
    for (int j = 0; j <= NY; j++)
      for (int i = 0; i < NX; i++) {
        size_t f = FYI(g, i, j, k);
        double mu = 0.0, eps = 0.0;
        if (j > 0 && j < NY) {
          if (o2)
            donor_flux2(W, 1, dy, dz * dx, W->dvy[f], CI(g, i, j - 1, k), CI(g, i, j, k), &mu, &eps);
          else
            donor_flux(W, W->dvy[f], CI(g, i, j - 1, k), CI(g, i, j, k), &mu, &eps);
        }
        W->muy[f] = mu; W->ey[f] = eps;
      }
#pragma omp parallel for schedule(static)
  for (int k = 0; k <= NZ; k++)
    for (int j = 0; j < NY; j++)
      for (int i = 0; i < NX; i++) {
        size_t f = FZI(g, i, j, k);
        double mu = 0.0, eps = 0.0;
        if (k > 0 && k < NZ) {
          if (o2)
            donor_flux2(W, 2, dz, dx * dy, W->dvz[f], CI(g, i, j, k - 1), CI(g, i, j, k), &mu, &eps);
          else
            donor_flux(W, W->dvz[f], CI(g, i, j, k - 1), CI(g, i, j, k), &mu, &eps);
        }
        W->muz[f] = mu; W->ez[f] = eps;
      }
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int k = 0; k < NZ; k++)
    for (int j = 0; j < NY; j++)
      for (int i = 0; i < NX; i++) {
        size_t c = CI(g, i, j, k);
        double netm = (W->mux[FXI(g, i + 1, j, k)] - W->mux[FXI(g, i, j, k)]) +
                      (W->muy[FYI(g, i, j + 1, k)] - W->muy[FYI(g, i, j, k)]) +
                      (W->muz[FZI(g, i, j, k + 1)] - W->muz[FZI(g, i, j, k)]);
        double nete = (W->ex[FXI(g, i + 1, j, k)] - W->ex[FXI(g, i, j, k)]) +
                      (W->ey[FYI(g, i, j + 1, k)] - W->ey[FYI(g, i, j, k)]) +
                      (W->ez[FZI(g, i, j, k + 1)] - W->ez[FZI(g, i, j, k)]);
        /* M_c = m_c - net mass outflow, E_c = m_c e^L_c - net energy outflow;
         * rho^{n+1} = M_c / V0 and e^pre = E_c / M_c are evaluated in the
         * equivalent forms rho_c - net/V0 and e^L + (e^L net_m - net_e)/M_c,
         * so that a cell with no net flux keeps rho and e^L bit for bit. */
        W->M[c] = W->mc[c] - netm;
        W->rn[c] = rho[c] - netm / V0;
        if (!(W->M[c] > 0.0) || !(W->rn[c] > 0.0)) { bad |= 1; W->epre[c] = 0.0; continue; }
        W->epre[c] = W->eL[c] + (W->eL[c] * netm - nete) / W->M[c];
      }
  return bad ? ORC_ENUMERIC : ORC_OK;
}

/* ------------------------------------------------------------------ */
/* O10: dual-mesh momentum and kinetic-energy remap at nodes            */
/* ------------------------------------------------------------------ */
/* mass flux of the dual face between node (i,j,k) and its +axis neighbour:
 * one eighth of the sum, over the existing cells that share that edge, of
 * the cell's lower plus upper face mass flux along the same axis. */
static double dual_flux(const orc_config *g, const orc_ws *W, int axis, int i, int j, int k) {
  double s = 0.0;
  for (int o2 = -1; o2 <= 0; o2++)
    for (int o1 = -1; o1 <= 0; o1++) {
      int ci = i, cj = j, ck = k;
      if (axis == 0) { cj += o1; ck += o2; }
      if (axis == 1) { ci += o1; ck += o2; }
      if (axis == 2) { ci += o1; cj += o2; }
      if (!cell_exists(g, ci, cj, ck)) continue;
      if (axis == 0) s += W->mux[FXI(g, ci, cj, ck)] + W->mux[FXI(g, ci + 1, cj, ck)];
      if (axis == 1) s += W->muy[FYI(g, ci, cj, ck)] + W->muy[FYI(g, ci, cj + 1, ck)];
      if (axis == 2) s += W->muz[FZI(g, ci, cj, ck)] + W->muz[FZI(g, ci, cj, ck + 1)];
    }
  return 0.125 * s;
}

/* swept volume of the dual face between node (i,j,k) and its +axis
 * neighbour (order 2): one eighth of the sum of the lower plus upper face
 * swept volumes of the same cells as in dual_flux */
static double dual_swept(const orc_config *g, const orc_ws *W, int axis, int i, int j, int k) {
  double s = 0.0;
  for (int o2 = -1; o2 <= 0; o2++)
    for (int o1 = -1; o1 <= 0; o1++) {
      int ci = i, cj = j, ck = k;
      if (axis == 0) { cj += o1; ck += o2; }
      if (axis == 1) { ci += o1; ck += o2; }
      if (axis == 2) { ci += o1; cj += o2; }
      if (!cell_exists(g, ci, cj, ck)) continue;
      if (axis == 0) s += W->dvx[FXI(g, ci, cj, ck)] + W->dvx[FXI(g, ci + 1, cj, ck)];
      if (axis == 1) s += W->dvy[FYI(g, ci, cj, ck)] + W->dvy[FYI(g, ci, cj + 1, ck)];
      if (axis == 2) s += W->dvz[FZI(g, ci, cj, ck)] + W->dvz[FZI(g, ci, cj, ck + 1)];
    }
  return 0.125 * s;
}

/* donor velocity of the edge from node (i,j,k) to its +axis neighbour with
 * mass flux phi: node u' (order 1), or its limited linear reconstruction
 * along the edge at the dual swept volume's centroid (order 2; slopes zero
 * at a node whose neighbour along the axis is outside the mesh) */
static void donor_velocity(const orc_config *g, const orc_ws *W, int axis, int i, int j, int k, double phi,
                           double out[3]) {
  const int di = axis == 0, dj = axis == 1, dk = axis == 2;
  const int ni = (phi > 0.0) ? i : i + di, nj = (phi > 0.0) ? j : j + dj, nk = (phi > 0.0) ? k : k + dk;
  const size_t dn = NI(g, ni, nj, nk);
  const double *u[3] = {W->u1, W->v1, W->w1};
  for (int m = 0; m < 3; m++) out[m] = u[m][dn];
  if (g->order != 2) return;
  double hs[3];
  spacing(g, &hs[0], &hs[1], &hs[2]);
  const double area = hs[(axis + 1) % 3] * hs[(axis + 2) % 3];
  /* the dual swept volume and the flux take the same sign convention */
  const double dvA = dual_swept(g, W, axis, i, j, k) / area;
  const double sgn_dvA = (phi > 0.0) ? fabs(dvA) : -fabs(dvA);
  if (!node_exists(g, ni - di, nj - dj, nk - dk) || !node_exists(g, ni + di, nj + dj, nk + dk)) return;
  const size_t nm = NI(g, ni - di, nj - dj, nk - dk), np = NI(g, ni + di, nj + dj, nk + dk);
  for (int m = 0; m < 3; m++) {
    const double sl = orc_vanleer((u[m][dn] - u[m][nm]) / hs[axis], (u[m][np] - u[m][dn]) / hs[axis]);
    out[m] = orc_donor_value(u[m][dn], sl, hs[axis], sgn_dvA);
  }
}

static int stage_node_remap(const orc_config *g, orc_ws *W) {
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int k = 0; k <= NZ; k++)
    for (int j = 0; j <= NY; j++)
      for (int i = 0; i <= NX; i++) {
        size_t n = NI(g, i, j, k);
        double m = W->mp[n];
        double u1 = W->u1[n], v1 = W->v1[n], w1 = W->w1[n];
        double P[3] = {m * u1, m * v1, m * w1};
        double K = 0.5 * m * (u1 * u1 + v1 * v1 + w1 * w1);
        for (int axis = 0; axis < 3; axis++) {
          int di = axis == 0, dj = axis == 1, dk = axis == 2;
          /* edge to the +axis neighbour: outflow from this node */
          if (node_exists(g, i + di, j + dj, k + dk)) {
            double phi = dual_flux(g, W, axis, i, j, k);
            double dv[3];
            donor_velocity(g, W, axis, i, j, k, phi, dv);
            double ud = dv[0], vd = dv[1], wd = dv[2];
            P[0] -= phi * ud; P[1] -= phi * vd; P[2] -= phi * wd;
            K -= phi * 0.5 * (ud * ud + vd * vd + wd * wd);
          }
          /* edge from the -axis neighbour: inflow to this node */
          if (node_exists(g, i - di, j - dj, k - dk)) {
            double phi = dual_flux(g, W, axis, i - di, j - dj, k - dk);
            double dv[3];
            donor_velocity(g, W, axis, i - di, j - dj, k - dk, phi, dv);
            double ud = dv[0], vd = dv[1], wd = dv[2];
            P[0] += phi * ud; P[1] += phi * vd; P[2] += phi * wd;
            K += phi * 0.5 * (ud * ud + vd * vd + wd * wd);
          }
        }
        double s = 0.0;
        for (int cc = -1; cc <= 0; cc++)
          for (int b = -1; b <= 0; b++)
            for (int a = -1; a <= 0; a++)
              if (cell_exists(g, i + a, j + b, k + cc)) s += W->M[CI(g, i + a, j + b, k + cc)];
        double mn = 0.125 * s;
        W->mn[n] = mn;
        if (!(mn > 0.0)) { bad |= 1; W->un[n] = W->vn[n] = W->wn[n] = 0.0; W->dK[n] = 0.0; continue; }
        double un = P[0] / mn, vn = P[1] / mn, wn = P[2] / mn;
        if (i == 0 || i == NX) un = 0.0;
        if (j == 0 || j == NY) vn = 0.0;
        if (k == 0 || k == NZ) wn = 0.0;
        W->un[n] = un; W->vn[n] = vn; W->wn[n] = wn;
        W->dK[n] = K - 0.5 * mn * (un * un + vn * vn + wn * wn);
      }
  return bad ? ORC_ENUMERIC : ORC_OK;
}

/* ------------------------------------------------------------------ */
/* O11 + O12: kinetic-energy fix and commit                             */
/* ------------------------------------------------------------------ */
static int stage_ke_fix_commit(const orc_config *g, orc_ws *W, double *rho, double *e,
                               double *u, double *v, double *w) {
  size_t nc = (size_t)NX * NY * NZ, nn = (size_t)(NX + 1) * (NY + 1) * (NZ + 1);
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int k = 0; k < NZ; k++)
    for (int j = 0; j < NY; j++)
      for (int i = 0; i < NX; i++) {
        size_t c = CI(g, i, j, k);
        double s = 0.0;
        for (int cc = 0; cc < 2; cc++)
          for (int b = 0; b < 2; b++)
            for (int a = 0; a < 2; a++) {
              size_t n = NI(g, i + a, j + b, k + cc);
              s += W->dK[n] / W->mn[n];
            }
        double en = W->epre[c] + 0.125 * s;
        if (!(en >= 0.0)) bad |= 1;
        W->E[c] = en; /* reuse as the new internal energy */
      }
  if (bad) return ORC_ENUMERIC;
  for (size_t c = 0; c < nc; c++) {
    rho[c] = W->rn[c];
    e[c] = W->E[c];
  }
  for (size_t n = 0; n < nn; n++) {
    u[n] = W->un[n]; v[n] = W->vn[n]; w[n] = W->wn[n];
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* public entry points                                                  */
/* ------------------------------------------------------------------ */

/* Time step of the current state (O3), clipped to t_end - t. */
/* Threads the OpenMP loops run on (the benchmark reports it beside the
 * oracle's timings), and a way to change it for the calling thread's later
 * loops (results do not depend on it). */
int orc_max_threads(void) { return omp_get_max_threads(); }
void orc_set_threads(int n) {
  if (n > 0) omp_set_num_threads(n);
}

int orc_timestep(const orc_config *g, orc_ws *W, const double *rho, const double *e,
                 const double *u, const double *v, const double *w, double t, double *dt_out) {
  if (!config_valid(g) || !W || W->nx != g->nx || W->ny != g->ny || W->nz != g->nz)
    return ORC_EINVAL;
  double dx, dy, dz;
  spacing(g, &dx, &dy, &dz);
  const double h = fmin(dx, fmin(dy, dz));
  if (!state_admissible(g, rho, e, u, v, w)) { *dt_out = NAN; return ORC_ENUMERIC; }
  stage_cells_eos_div_q(g, rho, e, u, v, w, W);
  double amax = stage_max_signal(g, u, v, w, W);
  if (!isfinite(amax)) { *dt_out = NAN; return ORC_ENUMERIC; }
  double rem = g->t_end - t;
  double dt = (amax > 0.0) ? g->cfl * h / amax : rem;
  if (!(dt <= rem)) dt = (dt > rem) ? rem : dt; /* NaN stays NaN */
  *dt_out = dt;
  if (!(isfinite(dt))) return ORC_ENUMERIC;
  return ORC_OK;
}

/* One Lagrange + remap step (O1..O12) in place on (rho, e, u, v, w, *t).
 * Returns ORC_DONE without touching the state if *t >= t_end; on an error
 * code the state is left as it was on entry. *dt_out receives the step. */
int orc_step(const orc_config *g, orc_ws *W, double *rho, double *e, double *u, double *v,
             double *w, double *t, double *dt_out) {
  if (!config_valid(g) || !W || W->nx != g->nx || W->ny != g->ny || W->nz != g->nz)
    return ORC_EINVAL;
  if (dt_out) *dt_out = 0.0;
  if (*t >= g->t_end) return ORC_DONE;
  double dt;
  int rc = orc_timestep(g, W, rho, e, u, v, w, *t, &dt); /* O1(m_c), O2, O4, O3 */
  if (rc != ORC_OK) return rc;
  if (!(dt > 0.0)) return ORC_ENUMERIC;
  stage_nodal_mass(g, W->mc, W->mp);                      /* O1 */
  if ((rc = stage_predictor(g, rho, e, dt, W)) != ORC_OK) return rc;   /* O5 */
  stage_forces_motion(g, u, v, w, dt, W);                 /* O6 */
  stage_compatible_energy(g, e, dt, W);                   /* O7 */
  if ((rc = stage_geometry(g, dt, W)) != ORC_OK) return rc;           /* O8 */
  if ((rc = stage_cell_remap(g, rho, W)) != ORC_OK) return rc;             /* O9 */
  if ((rc = stage_node_remap(g, W)) != ORC_OK) return rc;             /* O10 */
  if ((rc = stage_ke_fix_commit(g, W, rho, e, u, v, w)) != ORC_OK) return rc; /* O11 */
  *t = *t + dt;                                           /* O12 */
  if (dt_out) *dt_out = dt;
  return ORC_OK;
}

/* Pairwise sum (deterministic, error O(log n * eps)). */
static double pairwise_sum(const double *x, size_t n) {
  if (n <= 8) {
    double s = 0.0;
    for (size_t a = 0; a < n; a++) s += x[a];
    return s;
  }
  size_t h = n / 2;
  return pairwise_sum(x, h) + pairwise_sum(x + h, n - h);
}

/* Diagnostics: total mass sum(rho V0) and total energy
 * sum(rho V0 e) + sum(0.5 m_p |u_p|^2), m_p the nodal mass of O1. */
int orc_totals(const orc_config *g, const double *rho, const double *e, const double *u,
               const double *v, const double *w, double *mass, double *energy) {
  if (!config_valid(g)) return ORC_EINVAL;
  double dx, dy, dz;
  spacing(g, &dx, &dy, &dz);
  const double V0 = dx * dy * dz;
  size_t nc = (size_t)NX * NY * NZ, nn = (size_t)(NX + 1) * (NY + 1) * (NZ + 1);
  double *mc = (double *)malloc(nc * sizeof(double));
  double *ie = (double *)malloc(nc * sizeof(double));
  double *mp = (double *)malloc(nn * sizeof(double));
  double *ke = (double *)malloc(nn * sizeof(double));
  if (!mc || !ie || !mp || !ke) { free(mc); free(ie); free(mp); free(ke); return ORC_ENOMEM; }
  for (size_t c = 0; c < nc; c++) { mc[c] = rho[c] * V0; ie[c] = mc[c] * e[c]; }
  stage_nodal_mass(g, mc, mp);
  for (size_t n = 0; n < nn; n++) ke[n] = 0.5 * mp[n] * (u[n] * u[n] + v[n] * v[n] + w[n] * w[n]);
  *mass = pairwise_sum(mc, nc);
  *energy = pairwise_sum(ie, nc) + pairwise_sum(ke, nn);
  free(mc); free(ie); free(mp); free(ke);
  return ORC_OK;
}

/* Sod shock tube along x: a cell is "left" iff its centre x < x_split.
 * e = p / ((gamma-1) rho), u = 0. */
int orc_init_sod(const orc_config *g, double x_split, double rhoL, double pL, double rhoR,
                 double pR, double *rho, double *e, double *u, double *v, double *w) {
  if (!config_valid(g)) return ORC_EINVAL;
  double dx, dy, dz;
  spacing(g, &dx, &dy, &dz);
  for (int k = 0; k < NZ; k++)
    for (int j = 0; j < NY; j++)
      for (int i = 0; i < NX; i++) {
        size_t c = CI(g, i, j, k);
        double xc = g->lo[0] + (i + 0.5) * dx;
        int left = xc < x_split;
        rho[c] = left ? rhoL : rhoR;
        e[c] = (left ? pL : pR) / ((g->gamma - 1.0) * rho[c]);
      }
  size_t nn = (size_t)(NX + 1) * (NY + 1) * (NZ + 1);
  for (size_t n = 0; n < nn; n++) u[n] = v[n] = w[n] = 0.0;
  return ORC_OK;
}

/* Sedov blast in the octant: uniform rho0 with e = p0/((gamma-1) rho0); the
 * corner cell (0,0,0) holds the deposited energy as internal energy,
 * replacing its background value: e = E_dep / (rho0 V0). u = 0. */
int orc_init_sedov(const orc_config *g, double rho0, double p0, double edep, double *rho,
                   double *e, double *u, double *v, double *w) {
  if (!config_valid(g)) return ORC_EINVAL;
  double dx, dy, dz;
  spacing(g, &dx, &dy, &dz);
  const double V0 = dx * dy * dz;
  size_t nc = (size_t)NX * NY * NZ, nn = (size_t)(NX + 1) * (NY + 1) * (NZ + 1);
#pragma omp parallel for schedule(static)
  for (size_t c = 0; c < nc; c++) {
    rho[c] = rho0;
    e[c] = p0 / ((g->gamma - 1.0) * rho0);
  }
  e[0] = edep / (rho0 * V0);
#pragma omp parallel for schedule(static)
  for (size_t n = 0; n < nn; n++) u[n] = v[n] = w[n] = 0.0;
  return ORC_OK;
}

/* Noh implosion (the shock problem of Noh, 1987, that Sec. I-D lists among
 * the problems ScalSALE solves, in 1D, 2D or 3D): uniform rho0 with e = p0/((gamma-1) rho0) and every node
 * moving toward the corner lo at speed u0 along the first `dims` axes
 * (1 planar along x, 2 cylindrical about the z axis, 3 spherical): with
 * r = (i dx, j dy, k dz) restricted to those axes, u_p = -u0 r/|r| (zero at
 * r = 0). Wall-normal components are then zeroed on the six walls, as the
 * reflective walls require; the walls through lo are symmetry planes of the
 * problem, the others close the box. */
int orc_init_noh(const orc_config *g, double rho0, double p0, double u0, int dims, double *rho,
                 double *e, double *u, double *v, double *w) {
  if (!config_valid(g) || dims < 1 || dims > 3) return ORC_EINVAL;
  double dx, dy, dz;
  spacing(g, &dx, &dy, &dz);
  size_t nc = (size_t)NX * NY * NZ;
  for (size_t c = 0; c < nc; c++) {
    rho[c] = rho0;
    e[c] = p0 / ((g->gamma - 1.0) * rho0);
  }
  for (int k = 0; k <= NZ; k++)
    for (int j = 0; j <= NY; j++)
      for (int i = 0; i <= NX; i++) {
        double r[3] = {i * dx, dims >= 2 ? j * dy : 0.0, dims >= 3 ? k * dz : 0.0};
        double len = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
        double vel[3] = {0.0, 0.0, 0.0};
        if (len > 0.0)
          for (int a = 0; a < 3; a++) vel[a] = -u0 * (r[a] / len);
        if (i == 0 || i == NX) vel[0] = 0.0;
        if (j == 0 || j == NY) vel[1] = 0.0;
        if (k == 0 || k == NZ) vel[2] = 0.0;
        size_t n = NI(g, i, j, k);
        u[n] = vel[0];
        v[n] = vel[1];
        w[n] = vel[2];
      }
  return ORC_OK;
}

/* Run whole steps until t >= t_end or max_steps. Returns the last step's
 * code (ORC_DONE when t_end was reached); *steps counts completed steps. */
int orc_run(const orc_config *g, orc_ws *W, double *rho, double *e, double *u, double *v,
            double *w, double *t, int64_t max_steps, int64_t *steps) {
  int64_t n = 0;
  int rc = ORC_OK;
  while (n < max_steps) {
    double dt;
    rc = orc_step(g, W, rho, e, u, v, w, t, &dt);
    if (rc != ORC_OK) break;
    n++;
  }
  if (rc == ORC_OK && *t >= g->t_end) rc = ORC_DONE;
  if (steps) *steps = n;
  return rc;
}

/* O8 alone, for testing: given node displacements (dX, dY, dZ), return the
 * Lagrangian cell volumes V0 + sum_axes(dV_upper - dV_lower) in VL and the
 * face swept volumes in the workspace. Wall-normal displacement components on
 * wall nodes must be zero (as after O6); boundary faces are taken as zero. */
int orc_geometry(const orc_config *g, orc_ws *W, const double *dX, const double *dY,
                 const double *dZ, double *VL) {
  if (!config_valid(g) || !W || W->nx != g->nx || W->ny != g->ny || W->nz != g->nz)
    return ORC_EINVAL;
  size_t nc = (size_t)NX * NY * NZ, nn = (size_t)(NX + 1) * (NY + 1) * (NZ + 1);
  double dx, dy, dz;
  spacing(g, &dx, &dy, &dz);
  for (size_t n = 0; n < nn; n++) { W->ub[n] = dX[n]; W->vb[n] = dY[n]; W->wb[n] = dZ[n]; }
  for (size_t c = 0; c < nc; c++) W->mc[c] = dx * dy * dz; /* rho^L = 1 placeholder */
  int rc = stage_geometry(g, 1.0, W);
  for (size_t c = 0; c < nc; c++) VL[c] = W->VL[c];
  return rc;
}

/* Pressure p = (gamma-1) rho e and artificial viscosity q of a state (O2, O4),
 * for checking exported derived fields. */
int orc_derived(const orc_config *g, orc_ws *W, const double *rho, const double *e,
                const double *u, const double *v, const double *w, double *p, double *q) {
  if (!config_valid(g) || !W || W->nx != g->nx || W->ny != g->ny || W->nz != g->nz)
    return ORC_EINVAL;
  stage_cells_eos_div_q(g, rho, e, u, v, w, W);
  size_t nc = (size_t)NX * NY * NZ;
  for (size_t c = 0; c < nc; c++) { p[c] = W->p[c]; q[c] = W->q[c]; }
  return ORC_OK;
}
