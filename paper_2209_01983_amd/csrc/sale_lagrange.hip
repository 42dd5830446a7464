// sale_lagrange.hip -- the pure-Lagrangian step ("Lagrangian rezoning",
// ScalSALE Table I and Fig. 2a): the mesh moves with the flow and is never
// remapped. FP64 only. The paper prints no scheme; the kernels compute the
// project's FP64 oracle reading of it (its steps L1..L8):
//
//   k_lag_forces  L1, L2, L4, L5: geometry of each cell at t^n (exact volume
//                 and corner vectors dV/dx_a of the trilinear hex, length
//                 scale V / largest face area), EOS, divergence, viscosity,
//                 acoustic predictor P*, viscous hourglass forces; writes the
//                 8 corner forces of the cell
//   k_lag_nodes   L6: node force = gather of the corner forces of the node's
//                 cells (no atomics), u', walls, x' = x + dt (u + u')/2
//   k_lag_energy  L7, L8: compatible energy update, the new volume, density
//                 and admissibility, and the next step's signal a / h (max
//                 over cells into the control block)
//
// One thread per cell or node; the per-cell work is a few thousand FP64
// operations on data gathered from 8 nodes, so these kernels are bound by
// arithmetic, not by their ~0.5 KB per cell of HBM traffic.
#include "sale_device.h"

namespace sale {
namespace {

constexpr int TPL = 256;
inline int lag_blocks(int64_t n) { return (int)((n + TPL - 1) / TPL); }

__device__ __forceinline__ void ijk_of(int64_t q, int nx, int ny, int &i, int &j, int &k) {
  i = (int)(q % nx);
  const int64_t r = q / nx;
  j = (int)(r % ny);
  k = (int)(r / ny);
}
__device__ __forceinline__ int64_t node_at(const Mesh &m, int i, int j, int k) {
  return i + (int64_t)(m.nx + 1) * (j + (int64_t)(m.ny + 1) * k);
}

// Volume V and corner vectors S[a] = dV/dX[a] of the trilinear hex with
// corners X[a] (a = bits along x, y, z). With r = (r0, r1, r2) in the unit
// cube, the Jacobian columns are weighted sums of the cell's 4 edges along
// each axis, and det J is at most quadratic in each r_d, so the two-point
// Gauss rule per axis integrates det J and its derivative exactly.
__device__ void hex_volume(const double X[8][3], double S[8][3], double &V) {
  const double lo = 0.5 - 0.5 / sqrt(3.0), hi = 0.5 + 0.5 / sqrt(3.0);
#pragma unroll
  for (int a = 0; a < 8; a++) S[a][0] = S[a][1] = S[a][2] = 0.0;
  V = 0.0;
#pragma unroll 1  // one Gauss point at a time: fewer live registers
  for (int q = 0; q < 8; q++) {
    const double r0 = (q & 1) ? hi : lo, r1 = (q & 2) ? hi : lo, r2 = (q & 4) ? hi : lo;
    // weights of the four edges along each axis at this point
    // axis 0 edges: (0,1) (2,3) (4,5) (6,7), weights (1-r1)(1-r2), r1(1-r2), (1-r1)r2, r1 r2
    const double w0[4] = {(1 - r1) * (1 - r2), r1 * (1 - r2), (1 - r1) * r2, r1 * r2};
    // axis 1 edges: (0,2) (1,3) (4,6) (5,7), weights (1-r0)(1-r2), r0(1-r2), (1-r0)r2, r0 r2
    const double w1[4] = {(1 - r0) * (1 - r2), r0 * (1 - r2), (1 - r0) * r2, r0 * r2};
    // axis 2 edges: (0,4) (1,5) (2,6) (3,7), weights (1-r0)(1-r1), r0(1-r1), (1-r0)r1, r0 r1
    const double w2[4] = {(1 - r0) * (1 - r1), r0 * (1 - r1), (1 - r0) * r1, r0 * r1};
    double J[3][3];
#pragma unroll
    for (int c = 0; c < 3; c++) {
      J[0][c] = w0[0] * (X[1][c] - X[0][c]) + w0[1] * (X[3][c] - X[2][c]) + w0[2] * (X[5][c] - X[4][c]) +
                w0[3] * (X[7][c] - X[6][c]);
      J[1][c] = w1[0] * (X[2][c] - X[0][c]) + w1[1] * (X[3][c] - X[1][c]) + w1[2] * (X[6][c] - X[4][c]) +
                w1[3] * (X[7][c] - X[5][c]);
      J[2][c] = w2[0] * (X[4][c] - X[0][c]) + w2[1] * (X[5][c] - X[1][c]) + w2[2] * (X[6][c] - X[2][c]) +
                w2[3] * (X[7][c] - X[3][c]);
    }
    // cofactor columns: K[d] = J[d+1] x J[d+2]
    double K[3][3];
#pragma unroll
    for (int d = 0; d < 3; d++) {
      const double *A = J[(d + 1) % 3], *B = J[(d + 2) % 3];
      K[d][0] = A[1] * B[2] - A[2] * B[1];
      K[d][1] = A[2] * B[0] - A[0] * B[2];
      K[d][2] = A[0] * B[1] - A[1] * B[0];
    }
    V += 0.125 * (J[0][0] * K[0][0] + J[0][1] * K[0][1] + J[0][2] * K[0][2]);
    // dJ[d]/dX[a] = +w or -w of the edge along d that has corner a at its upper or lower end
#pragma unroll
    for (int a = 0; a < 8; a++) {
      const int b0 = a & 1, b1 = (a >> 1) & 1, b2 = (a >> 2) & 1;
      const double g0 = (b0 ? 1.0 : -1.0) * w0[b1 + 2 * b2];
      const double g1 = (b1 ? 1.0 : -1.0) * w1[b0 + 2 * b2];
      const double g2 = (b2 ? 1.0 : -1.0) * w2[b0 + 2 * b1];
#pragma unroll
      for (int c = 0; c < 3; c++) S[a][c] += 0.125 * (g0 * K[0][c] + g1 * K[1][c] + g2 * K[2][c]);
    }
  }
}

// V / (largest face area), a face's area being half the norm of the cross
// product of its diagonals
__device__ double length_scale(const double X[8][3], double V) {
  // faces as corner cycles: x-, x+, y-, y+, z-, z+
  const int F[6][4] = {{0, 2, 6, 4}, {1, 3, 7, 5}, {0, 1, 5, 4}, {2, 3, 7, 6}, {0, 1, 3, 2}, {4, 5, 7, 6}};
  double amax = 0.0;
#pragma unroll
  for (int f = 0; f < 6; f++) {
    double p[3], q[3];
#pragma unroll
    for (int c = 0; c < 3; c++) {
      p[c] = X[F[f][2]][c] - X[F[f][0]][c];
      q[c] = X[F[f][3]][c] - X[F[f][1]][c];
    }
    const double nx = p[1] * q[2] - p[2] * q[1], ny = p[2] * q[0] - p[0] * q[2], nz = p[0] * q[1] - p[1] * q[0];
    amax = fmax(amax, 0.5 * sqrt(nx * nx + ny * ny + nz * nz));
  }
  return V / amax;
}

__device__ __forceinline__ void load_corners(const Mesh &m, const double *a0, const double *a1, const double *a2,
                                             int i, int j, int k, double X[8][3]) {
#pragma unroll
  for (int a = 0; a < 8; a++) {
    const int64_t n = node_at(m, i + (a & 1), j + ((a >> 1) & 1), k + ((a >> 2) & 1));
    X[a][0] = a0[n];
    X[a][1] = a1[n];
    X[a][2] = a2[n];
  }
}

// divergence, largest node speed and signal a / h of a cell (L2, L3)
struct CellKin {
  double D, smax;
};
__device__ __forceinline__ CellKin kinematics(const double S[8][3], const double U[8][3], double V) {
  double div = 0.0, smax = 0.0;
#pragma unroll
  for (int a = 0; a < 8; a++) {
    div += S[a][0] * U[a][0] + S[a][1] * U[a][1] + S[a][2] * U[a][2];
    smax = fmax(smax, sqrt(U[a][0] * U[a][0] + U[a][1] * U[a][1] + U[a][2] * U[a][2]));
  }
  return {div / V, smax};
}

__global__ void k_lag_begin(Mesh m, Ctl *ctl) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (ctl->status != 0u || ctl->t >= ctl->t_end) {
    ctl->done = 1u;
    return;
  }
  const double r = __longlong_as_double((long long)ctl->amax_bits);  // max over cells of a / h
  const double rem = ctl->t_end - ctl->t;
  double dt = r > 0.0 ? m.cfl / r : rem;
  if (dt > rem) dt = rem;
  if (!(dt > 0.0) || !isfinite(dt)) {
    ctl->status |= SALE_FLAG_NUMERIC;
    ctl->done = 1u;
    return;
  }
  ctl->dt = dt;
  ctl->done = 0u;
  ctl->t = ctl->t + dt;
  ctl->step += 1;
  ctl->amax_bits = 0ull;
}

__global__ __launch_bounds__(TPL) void k_lag_forces(Mesh m, Ctl *ctl, State<double> cur, const double *x,
                                                    const double *y, const double *z, const double *mass,
                                                    double *F) {
  if (ctl->done) return;
  const int64_t c = blockIdx.x * (int64_t)TPL + threadIdx.x;
  if (c >= m.ncell) return;
  int i, j, k;
  ijk_of(c, m.nx, m.ny, i, j, k);
  const double dt = ctl->dt;
  const int64_t fs = corner_stride(m.ncell);
  double X[8][3], S[8][3], V;
  load_corners(m, x, y, z, i, j, k, X);
  hex_volume(X, S, V);
  double Fc[8][3];
  bool ok = V > 0.0;
  if (ok) {
    double U[8][3];
    load_corners(m, cur.u, cur.v, cur.w, i, j, k, U);
    const double h = length_scale(X, V);
    const double mc = mass[c], e = cur.e[c];
    const double rho = mc / V;
    const double p = m.gm1 * rho * e;
    const double cs = sqrt(m.ggm1 * fmax(e, 0.0));
    const CellKin kin = kinematics(S, U, V);
    double q = 0.0;
    if (kin.D < 0.0) {
      const double hd = h * kin.D;
      q = rho * (m.cq * hd * hd + m.cl * cs * h * fabs(kin.D));
    }
    const double dVs = 0.5 * dt * V * kin.D;
    const double Vs = V + dVs;
    ok = Vs > 0.0;
    const double Ps = m.gm1 * (mc / Vs) * (e - (p + q) * dVs / mc) + q;
    // viscous hourglass forces on the four hourglass patterns, each made
    // orthogonal to linear velocity fields on this cell's shape
    const double coef = m.chg * rho * cs * cbrt(V * V);
#pragma unroll
    for (int a = 0; a < 8; a++)
#pragma unroll
      for (int d = 0; d < 3; d++) Fc[a][d] = Ps * S[a][d];
#pragma unroll
    for (int hk = 0; hk < 4; hk++) {
      double G[8];
#pragma unroll
      for (int a = 0; a < 8; a++) {
        const double sx = (a & 1) ? 1.0 : -1.0, sy = (a & 2) ? 1.0 : -1.0, sz = (a & 4) ? 1.0 : -1.0;
        G[a] = hk == 0 ? sy * sz : hk == 1 ? sz * sx : hk == 2 ? sx * sy : sx * sy * sz;
      }
      double hx[3] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int a = 0; a < 8; a++)
#pragma unroll
        for (int d = 0; d < 3; d++) hx[d] += G[a] * X[a][d];
      double gam[8], g[3] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int a = 0; a < 8; a++) {
        gam[a] = G[a] - (hx[0] * S[a][0] + hx[1] * S[a][1] + hx[2] * S[a][2]) / V;
#pragma unroll
        for (int d = 0; d < 3; d++) g[d] += gam[a] * U[a][d];
      }
#pragma unroll
      for (int a = 0; a < 8; a++)
#pragma unroll
        for (int d = 0; d < 3; d++) Fc[a][d] -= coef * gam[a] * g[d];
    }
  }
  if (!ok) {
    atomicOr(&ctl->status, SALE_FLAG_TANGLE);
#pragma unroll
    for (int a = 0; a < 8; a++) Fc[a][0] = Fc[a][1] = Fc[a][2] = 0.0;
  }
#pragma unroll
  for (int a = 0; a < 8; a++)
#pragma unroll
    for (int d = 0; d < 3; d++) F[(3 * a + d) * fs + c] = Fc[a][d];
}

__global__ __launch_bounds__(TPL) void k_lag_nodes(Mesh m, Ctl *ctl, State<double> cur, State<double> nxt,
                                                   const double *x0, const double *y0, const double *z0, double *x1,
                                                   double *y1, double *z1, const double *mass, const double *F) {
  const int64_t n = blockIdx.x * (int64_t)TPL + threadIdx.x;
  if (n >= m.nnode) return;
  if (ctl->done) {  // no-op step: carry the nodes across
    nxt.u[n] = cur.u[n], nxt.v[n] = cur.v[n], nxt.w[n] = cur.w[n];
    x1[n] = x0[n], y1[n] = y0[n], z1[n] = z0[n];
    return;
  }
  int i, j, k;
  ijk_of(n, m.nx + 1, m.ny + 1, i, j, k);
  const int64_t fs = corner_stride(m.ncell);
  double f[3] = {0.0, 0.0, 0.0}, ms = 0.0;
#pragma unroll
  for (int a = 0; a < 8; a++) {  // this node is corner a of cell (i, j, k) - bits(a)
    const int ci = i - (a & 1), cj = j - ((a >> 1) & 1), ck = k - ((a >> 2) & 1);
    if (ci < 0 || ci >= m.nx || cj < 0 || cj >= m.ny || ck < 0 || ck >= m.nz) continue;
    const int64_t c = ci + (int64_t)m.nx * (cj + (int64_t)m.ny * ck);
#pragma unroll
    for (int d = 0; d < 3; d++) f[d] += F[(3 * a + d) * fs + c];
    ms += mass[c];
  }
  const double mp = 0.125 * ms, dt = ctl->dt;
  const double uo[3] = {cur.u[n], cur.v[n], cur.w[n]};
  double un[3];
#pragma unroll
  for (int d = 0; d < 3; d++) un[d] = uo[d] + dt * f[d] / mp;
  if (i == 0 || i == m.nx) un[0] = 0.0;
  if (j == 0 || j == m.ny) un[1] = 0.0;
  if (k == 0 || k == m.nz) un[2] = 0.0;
  nxt.u[n] = un[0], nxt.v[n] = un[1], nxt.w[n] = un[2];
  x1[n] = x0[n] + dt * (0.5 * (uo[0] + un[0]));
  y1[n] = y0[n] + dt * (0.5 * (uo[1] + un[1]));
  z1[n] = z0[n] + dt * (0.5 * (uo[2] + un[2]));
}

// the signal a / h of one cell from its geometry (positions X, corner
// vectors S, volume V > 0), node velocities U and energy e
__device__ double signal_of(const Mesh &m, const double X[8][3], const double S[8][3], double V,
                            const double U[8][3], double e) {
  const double h = length_scale(X, V);
  const double cs = sqrt(m.ggm1 * fmax(e, 0.0));
  const CellKin kin = kinematics(S, U, V);
  const double a = cs + kin.smax + 4.0 * m.cq * h * fmax(-kin.D, 0.0);
  return a / h;
}

template <int NT>
__device__ __forceinline__ void flags_and_max(Ctl *ctl, double r, bool tangled, bool numeric) {
  __shared__ double red[NT / 64];
  __shared__ unsigned int flags;
  if (threadIdx.x == 0) flags = 0u;
  __syncthreads();
  if (tangled) atomicOr(&flags, SALE_FLAG_TANGLE);
  if (numeric) atomicOr(&flags, SALE_FLAG_NUMERIC);
  r = wave_max(r);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = r;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = red[0];
    for (int q = 1; q < NT / 64; q++) b = fmax(b, red[q]);
    if (b > 0.0) atomicMax(&ctl->amax_bits, (unsigned long long)__double_as_longlong(b));
    if (flags) atomicOr(&ctl->status, flags);
  }
}

__global__ __launch_bounds__(TPL) void k_lag_energy(Mesh m, Ctl *ctl, State<double> cur, State<double> nxt,
                                                    const double *x1, const double *y1, const double *z1,
                                                    const double *mass, const double *F) {
  const int64_t c = blockIdx.x * (int64_t)TPL + threadIdx.x;
  const bool live = c < m.ncell;
  if (ctl->done) {  // no-op step: carry the cells across
    if (live) nxt.rho[c] = cur.rho[c], nxt.e[c] = cur.e[c];
    return;
  }
  double r = 0.0;
  bool tangled = false, numeric = false;
  if (live) {
    int i, j, k;
    ijk_of(c, m.nx, m.ny, i, j, k);
    const double dt = ctl->dt, mc = mass[c];
    const int64_t fs = corner_stride(m.ncell);
    double work = 0.0;
#pragma unroll 1
    for (int a = 0; a < 8; a++) {
      const int64_t n = node_at(m, i + (a & 1), j + ((a >> 1) & 1), k + ((a >> 2) & 1));
      const double ub[3] = {0.5 * (cur.u[n] + nxt.u[n]), 0.5 * (cur.v[n] + nxt.v[n]), 0.5 * (cur.w[n] + nxt.w[n])};
#pragma unroll
      for (int d = 0; d < 3; d++) work += F[(3 * a + d) * fs + c] * ub[d];
    }
    const double en = cur.e[c] - dt * work / mc;
    double X[8][3], S[8][3], V;
    load_corners(m, x1, y1, z1, i, j, k, X);
    hex_volume(X, S, V);
    nxt.e[c] = en;
    nxt.rho[c] = mc / V;
    if (!(V > 0.0)) tangled = true;
    if (!isfinite(en) || !(en >= 0.0)) numeric = true;
    if (!tangled && !numeric) {
      double U[8][3];
      load_corners(m, nxt.u, nxt.v, nxt.w, i, j, k, U);
      r = signal_of(m, X, S, V, U, en);
      if (!isfinite(r)) numeric = true, r = 0.0;
    }
  }
  flags_and_max<TPL>(ctl, r, tangled, numeric);
}

// initial positions of the Cartesian mesh (products and sums rounded one by
// one, lo + i dx) and cell masses rho V0
__global__ __launch_bounds__(TPL) void k_lag_init_nodes(Mesh m, double *x, double *y, double *z) {
  const int64_t n = blockIdx.x * (int64_t)TPL + threadIdx.x;
  if (n >= m.nnode) return;
  int i, j, k;
  ijk_of(n, m.nx + 1, m.ny + 1, i, j, k);
  x[n] = m.lo[0] + mul_rn(i, m.dx);
  y[n] = m.lo[1] + mul_rn(j, m.dy);
  z[n] = m.lo[2] + mul_rn(k, m.dz);
}

__global__ __launch_bounds__(TPL) void k_lag_init_cells(Mesh m, Ctl *ctl, State<double> s, const double *x,
                                                        const double *y, const double *z, double *mass) {
  const int64_t c = blockIdx.x * (int64_t)TPL + threadIdx.x;
  const bool live = c < m.ncell;
  double r = 0.0;
  bool tangled = false;
  if (live) {
    mass[c] = s.rho[c] * m.V0;
    int i, j, k;
    ijk_of(c, m.nx, m.ny, i, j, k);
    double X[8][3], U[8][3], S[8][3], V;
    load_corners(m, x, y, z, i, j, k, X);
    load_corners(m, s.u, s.v, s.w, i, j, k, U);
    hex_volume(X, S, V);
    if (V > 0.0)
      r = signal_of(m, X, S, V, U, s.e[c]);
    else
      tangled = true;
  }
  flags_and_max<TPL>(ctl, r, tangled, false);
}

__global__ void k_lag_reset_signal(Ctl *ctl) {
  if (threadIdx.x == 0 && blockIdx.x == 0) ctl->amax_bits = 0ull;
}

__global__ __launch_bounds__(TPL) void k_fixed_positions(Mesh m, int axis, double *out) {
  const int64_t n = blockIdx.x * (int64_t)TPL + threadIdx.x;
  if (n >= m.nnode) return;
  int i, j, k;
  ijk_of(n, m.nx + 1, m.ny + 1, i, j, k);
  out[n] = axis == 0 ? m.lo[0] + mul_rn(i, m.dx) : axis == 1 ? m.lo[1] + mul_rn(j, m.dy) : m.lo[2] + mul_rn(k, m.dz);
}

}  // namespace

hipError_t launch_lag_init(const Mesh &m, Ctl *ctl, const Work<double> &w, hipStream_t s) {
  hipLaunchKernelGGL(k_lag_init_nodes, dim3(lag_blocks(m.nnode)), dim3(TPL), 0, s, m, w.lg.x[0], w.lg.y[0],
                     w.lg.z[0]);
  hipLaunchKernelGGL(k_lag_reset_signal, dim3(1), dim3(64), 0, s, ctl);
  hipLaunchKernelGGL(k_lag_init_cells, dim3(lag_blocks(m.ncell)), dim3(TPL), 0, s, m, ctl, w.s[0], w.lg.x[0],
                     w.lg.y[0], w.lg.z[0], w.lg.m);
  return hipGetLastError();
}

hipError_t launch_lag_step(const Mesh &m, Ctl *ctl, const Work<double> &w, int cur, hipStream_t s,
                           const hipEvent_t *ev) {
  const int nx = 1 - cur;
  hipError_t e = hipSuccess;
  if (ev) e = hipEventRecord(ev[0], s);
  hipLaunchKernelGGL(k_lag_begin, dim3(1), dim3(64), 0, s, m, ctl);
  if (ev && e == hipSuccess) e = hipEventRecord(ev[1], s);
  hipLaunchKernelGGL(k_lag_forces, dim3(lag_blocks(m.ncell)), dim3(TPL), 0, s, m, ctl, w.s[cur], w.lg.x[cur],
                     w.lg.y[cur], w.lg.z[cur], w.lg.m, w.lg.F);
  hipLaunchKernelGGL(k_lag_nodes, dim3(lag_blocks(m.nnode)), dim3(TPL), 0, s, m, ctl, w.s[cur], w.s[nx],
                     w.lg.x[cur], w.lg.y[cur], w.lg.z[cur], w.lg.x[nx], w.lg.y[nx], w.lg.z[nx], w.lg.m, w.lg.F);
  if (ev && e == hipSuccess) e = hipEventRecord(ev[2], s);
  hipLaunchKernelGGL(k_lag_energy, dim3(lag_blocks(m.ncell)), dim3(TPL), 0, s, m, ctl, w.s[cur], w.s[nx],
                     w.lg.x[nx], w.lg.y[nx], w.lg.z[nx], w.lg.m, w.lg.F);
  if (ev && e == hipSuccess) e = hipEventRecord(ev[3], s);
  const hipError_t l = hipGetLastError();
  return l != hipSuccess ? l : e;
}

template <typename R>
hipError_t launch_positions(const Mesh &m, const Work<R> &w, int cur, int axis, double *out, hipStream_t s) {
  if (m.mode == 1) {
    const double *src = axis == 0 ? w.lg.x[cur] : axis == 1 ? w.lg.y[cur] : w.lg.z[cur];
    return hipMemcpyAsync(out, src, (size_t)m.nnode * sizeof(double), hipMemcpyDeviceToDevice, s);
  }
  hipLaunchKernelGGL(k_fixed_positions, dim3(lag_blocks(m.nnode)), dim3(TPL), 0, s, m, axis, out);
  return hipGetLastError();
}
template hipError_t launch_positions<double>(const Mesh &, const Work<double> &, int, int, double *, hipStream_t);
template hipError_t launch_positions<float>(const Mesh &, const Work<float> &, int, int, double *, hipStream_t);

}  // namespace sale
