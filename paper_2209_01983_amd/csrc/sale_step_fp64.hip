// sale_step_fp64.hip -- FP64 SALE step for gfx950, multi-pass form.
//
// One step = the Lagrangian phase on the structured hex mesh followed by the
// Eulerian rezone and donor-cell advection back to the fixed mesh (ScalSALE
// Sec. I-D and Table I: "Lagrangian rezoning", "Eulerian rezoning",
// "Advection"), ideal-gas EoS (Sec. I-C/I-D), cell-centred rho/e/p/q and
// vertex velocities (Sec. III-B/III-C), density from mass over volume
// (Sec. III-A). The paper prints no scheme equations; the kernels compute the
// scheme of the project's FP64 oracle, stage by stage:
//   k_begin      O3  dt from the previous step's max signal speed, clipped to t_end
//   k_predict    O1/O2/O4/O5  EOS, divergence, viscosity, acoustic predictor P*
//   k_accel      O6  gather of corner forces (no atomics), u', walls
//   k_swept      O8  swept volumes of every cell's three lower faces (closed form)
//   k_lagr       O7/O8  compatible energy e^L, V^L, rho^L
//   k_flux       O9  donor mass / energy fluxes of the lower faces
//   k_remap      O9  M, rho^{n+1}, e^pre
//   k_node_remap O10 dual-mesh momentum/KE remap, u^{n+1} (in place), dK/m
//   k_finish     O11 KE fix, new state, next signal speed (wave-shuffle max)
// Every node-centred kernel gathers from its <= 8 cells; nothing scatters, so
// results do not depend on scheduling.
#include <math.h>

#include "../../include/sale.h"
#include "sale_impl.h"

namespace sale {
namespace {

constexpr int TPB = 256;

__device__ __forceinline__ int64_t cidx(const Mesh &m, int i, int j, int k) {
  return i + (int64_t)m.nx * (j + (int64_t)m.ny * k);
}
__device__ __forceinline__ int64_t nidx(const Mesh &m, int i, int j, int k) {
  return i + (int64_t)(m.nx + 1) * (j + (int64_t)(m.ny + 1) * k);
}
__device__ __forceinline__ void cell_ijk(const Mesh &m, int64_t c, int &i, int &j, int &k) {
  i = (int)(c % m.nx);
  int64_t r = c / m.nx;
  j = (int)(r % m.ny);
  k = (int)(r / m.ny);
}
__device__ __forceinline__ void node_ijk(const Mesh &m, int64_t n, int &i, int &j, int &k) {
  i = (int)(n % (m.nx + 1));
  int64_t r = n / (m.nx + 1);
  j = (int)(r % (m.ny + 1));
  k = (int)(r / (m.ny + 1));
}
__device__ __forceinline__ bool cell_in(const Mesh &m, int i, int j, int k) {
  return i >= 0 && i < m.nx && j >= 0 && j < m.ny && k >= 0 && k < m.nz;
}

// sum_p S_{c,p} . X_p over the 8 corners of cell (i,j,k), grouped as
// differences across the cell along each axis (+side minus -side of the same
// edge), scaled by the quarter face areas.
template <typename F>
__device__ __forceinline__ double corner_sum(const Mesh &m, int i, int j, int k, F X) {
  const int64_t sy = m.nx + 1, sz = (int64_t)(m.nx + 1) * (m.ny + 1);
  const int64_t n0 = nidx(m, i, j, k);
  double sx = 0.0, sy_ = 0.0, sz_ = 0.0;
#pragma unroll
  for (int t2 = 0; t2 < 2; t2++)
#pragma unroll
    for (int t1 = 0; t1 < 2; t1++) {
      sx += X(0, n0 + 1 + t1 * sy + t2 * sz) - X(0, n0 + t1 * sy + t2 * sz);
      sy_ += X(1, n0 + sy + t1 + t2 * sz) - X(1, n0 + t1 + t2 * sz);
      sz_ += X(2, n0 + sz + t1 + t2 * sy) - X(2, n0 + t1 + t2 * sy);
    }
  return m.ax * sx + m.ay * sy_ + m.az * sz_;
}

// Exact volume swept by a rectangular face (edge lengths h1 along its first
// tangent s, h2 along its second t; tangents cyclic after the normal) whose
// corners (s,t) = (0,0), (1,0), (0,1), (1,1) move by d0..d3, components
// (normal, t1, t2). With delta(s,t) = A + B s + C t + E s t:
//   V = h1 h2 <xi> + h1/2 <xi zeta_t - zeta xi_t> + h2/2 <xi eta_s - eta xi_s>
//       + 1/3 <delta . (delta_s x delta_t)>,  <.> = integral over [0,1]^2.
// The middle brackets reduce to 1D integrals along the edges t = 0 and
// s = 0 (their st terms cancel), and the triple product integrates to
//   A.(B x C) + 1/2 A.((B - C) x E) + 1/4 C.(B x E).
__device__ __forceinline__ double swept_volume(const double d0[3], const double d1[3],
                                               const double d2[3], const double d3[3],
                                               double h1, double h2) {
  double A[3], B[3], C[3], E[3];
#pragma unroll
  for (int a = 0; a < 3; a++) {
    A[a] = d0[a];
    B[a] = d1[a] - d0[a];
    C[a] = d2[a] - d0[a];
    E[a] = (d3[a] - d1[a]) - (d2[a] - d0[a]);
  }
  const double third = 1.0 / 3.0;
  const double t0 = h1 * h2 * (0.25 * ((d0[0] + d1[0]) + (d2[0] + d3[0])));
  // <xi zeta_t - zeta xi_t> = int_0^1 (A0 + B0 s)(C2 + E2 s) - (A2 + B2 s)(C0 + E0 s) ds
  const double i1 = (A[0] * C[2] + 0.5 * (A[0] * E[2] + B[0] * C[2]) + third * B[0] * E[2]) -
                    (A[2] * C[0] + 0.5 * (A[2] * E[0] + B[2] * C[0]) + third * B[2] * E[0]);
  // <xi eta_s - eta xi_s> = int_0^1 (A0 + C0 t)(B1 + E1 t) - (A1 + C1 t)(B0 + E0 t) dt
  const double i2 = (A[0] * B[1] + 0.5 * (A[0] * E[1] + C[0] * B[1]) + third * C[0] * E[1]) -
                    (A[1] * B[0] + 0.5 * (A[1] * E[0] + C[1] * B[0]) + third * C[1] * E[0]);
  double BC[3] = {B[1] * C[2] - B[2] * C[1], B[2] * C[0] - B[0] * C[2], B[0] * C[1] - B[1] * C[0]};
  double D_[3] = {B[0] - C[0], B[1] - C[1], B[2] - C[2]};
  double DE[3] = {D_[1] * E[2] - D_[2] * E[1], D_[2] * E[0] - D_[0] * E[2],
                  D_[0] * E[1] - D_[1] * E[0]};
  double BE[3] = {B[1] * E[2] - B[2] * E[1], B[2] * E[0] - B[0] * E[2], B[0] * E[1] - B[1] * E[0]};
  const double trip = (A[0] * BC[0] + A[1] * BC[1] + A[2] * BC[2]) +
                      0.5 * (A[0] * DE[0] + A[1] * DE[1] + A[2] * DE[2]) +
                      0.25 * (C[0] * BE[0] + C[1] * BE[1] + C[2] * BE[2]);
  return t0 + 0.5 * h1 * i1 + 0.5 * h2 * i2 + third * trip;
}

// ---- block reductions (wave64 shuffles, then LDS across the 4 waves) -------
__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
  return x;
}
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Signal speed a_c = c + max_p |u_p| + 4 C_Q h max(-D, 0) of cell (i,j,k) of
// the state (rho, e, u); raises NUMERIC for an inadmissible cell.
__device__ __forceinline__ double signal_speed(const Mesh &m, int i, int j, int k, double rho,
                                               double e, const double *u, const double *v,
                                               const double *w, bool &bad) {
  const double D =
      corner_sum(m, i, j, k, [&](int a, int64_t n) { return a == 0 ? u[n] : (a == 1 ? v[n] : w[n]); }) /
      m.V0;
  const double cs = sqrt(m.gamma * (m.gamma - 1.0) * fmax(e, 0.0));
  double s = 0.0;
#pragma unroll
  for (int cc = 0; cc < 2; cc++)
#pragma unroll
    for (int b = 0; b < 2; b++)
#pragma unroll
      for (int a = 0; a < 2; a++) {
        const int64_t n = nidx(m, i + a, j + b, k + cc);
        const double sp = sqrt(u[n] * u[n] + v[n] * v[n] + w[n] * w[n]);
        if (sp > s) s = sp;
        if (!isfinite(sp)) bad = true;
      }
  const double ac = cs + s + 4.0 * m.cq * m.h * fmax(-D, 0.0);
  if (!(rho > 0.0) || !isfinite(rho) || !(e >= 0.0) || !isfinite(e) || !isfinite(ac)) bad = true;
  return ac;
}

__device__ __forceinline__ void block_max_to_ctl(Ctl *ctl, double a, bool bad) {
  __shared__ double red[TPB / 64];
  __shared__ int anybad;
  if (threadIdx.x == 0) anybad = 0;
  __syncthreads();
  if (bad) anybad = 1;
  a = wave_max(bad ? 0.0 : a);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = red[0];
    for (int q = 1; q < TPB / 64; q++) r = fmax(r, red[q]);
    // a >= 0: the bit patterns of non-negative doubles order like the values
    if (r > 0.0) atomicMax(&ctl->amax_bits, (unsigned long long)__double_as_longlong(r));
    if (anybad) atomicOr(&ctl->status, SALE_FLAG_NUMERIC);
  }
}

// ---- step kernels -----------------------------------------------------------
__global__ void k_begin(Mesh m, Ctl *ctl) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (ctl->status != 0u || ctl->t >= ctl->t_end) {
    ctl->done = 1u;
    return;
  }
  const double amax = __longlong_as_double((long long)ctl->amax_bits);
  const double rem = ctl->t_end - ctl->t;
  double dt = amax > 0.0 ? m.cfl * m.h / amax : rem;
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

__global__ __launch_bounds__(TPB) void k_predict(Mesh m, Ctl *ctl, Fields64 f) {
  if (ctl->done) return;
  const int64_t c = blockIdx.x * (int64_t)TPB + threadIdx.x;
  if (c >= m.ncell) return;
  int i, j, k;
  cell_ijk(m, c, i, j, k);
  const double dt = ctl->dt;
  const double rho = f.rho[c], e = f.e[c];
  const double mc = rho * m.V0;
  const double p = (m.gamma - 1.0) * rho * e;
  const double cs = sqrt(m.gamma * (m.gamma - 1.0) * fmax(e, 0.0));
  const double D = corner_sum(m, i, j, k, [&](int a, int64_t n) {
                     return a == 0 ? f.u[n] : (a == 1 ? f.v[n] : f.w[n]);
                   }) / m.V0;
  double q = 0.0;
  if (D < 0.0) {
    const double hd = m.h * D;
    q = rho * (m.cq * hd * hd + m.cl * cs * m.h * fabs(D));
  }
  const double dVs = 0.5 * dt * m.V0 * D;
  const double Vs = m.V0 + dVs;
  if (!(Vs > 0.0)) {
    atomicOr(&ctl->status, SALE_FLAG_TANGLE);
    f.ps[c] = 0.0;
    return;
  }
  const double rs = mc / Vs;
  const double es = e - (p + q) * dVs / mc;
  f.ps[c] = (m.gamma - 1.0) * rs * es + q;
}

__global__ __launch_bounds__(TPB) void k_accel(Mesh m, Ctl *ctl, Fields64 f) {
  if (ctl->done) return;
  const int64_t n = blockIdx.x * (int64_t)TPB + threadIdx.x;
  if (n >= m.nnode) return;
  int i, j, k;
  node_ijk(m, n, i, j, k);
  const double dt = ctl->dt;
  double sm = 0.0;
  for (int cc = -1; cc <= 0; cc++)
    for (int b = -1; b <= 0; b++)
      for (int a = -1; a <= 0; a++)
        if (cell_in(m, i + a, j + b, k + cc)) sm += f.rho[cidx(m, i + a, j + b, k + cc)] * m.V0;
  const double mp = 0.125 * sm;
  auto P = [&](int ci, int cj, int ck) { return cell_in(m, ci, cj, ck) ? f.ps[cidx(m, ci, cj, ck)] : 0.0; };
  double F0 = 0.0, F1 = 0.0, F2 = 0.0;
#pragma unroll
  for (int t2 = 0; t2 < 2; t2++)
#pragma unroll
    for (int t1 = 0; t1 < 2; t1++) {
      F0 += P(i - 1, j - t1, k - t2) - P(i, j - t1, k - t2);
      F1 += P(i - t1, j - 1, k - t2) - P(i - t1, j, k - t2);
      F2 += P(i - t1, j - t2, k - 1) - P(i - t1, j - t2, k);
    }
  F0 *= m.ax;
  F1 *= m.ay;
  F2 *= m.az;
  double u1 = f.u[n] + dt * F0 / mp;
  double v1 = f.v[n] + dt * F1 / mp;
  double w1 = f.w[n] + dt * F2 / mp;
  if (i == 0 || i == m.nx) u1 = 0.0;
  if (j == 0 || j == m.ny) v1 = 0.0;
  if (k == 0 || k == m.nz) w1 = 0.0;
  f.u1[n] = u1;
  f.v1[n] = v1;
  f.w1[n] = w1;
}

// node displacement delta = dt * (u + u') / 2, components (x, y, z)
__device__ __forceinline__ void disp(const Fields64 &f, int64_t n, double dt, double d[3]) {
  d[0] = dt * (0.5 * (f.u[n] + f.u1[n]));
  d[1] = dt * (0.5 * (f.v[n] + f.v1[n]));
  d[2] = dt * (0.5 * (f.w[n] + f.w1[n]));
}

__global__ __launch_bounds__(TPB) void k_swept(Mesh m, Ctl *ctl, Fields64 f) {
  if (ctl->done) return;
  const int64_t c = blockIdx.x * (int64_t)TPB + threadIdx.x;
  if (c >= m.ncell) return;
  int i, j, k;
  cell_ijk(m, c, i, j, k);
  const double dt = ctl->dt;
  double g[4][3], d[4][3];
  // x face at node plane i: corner (s,t) -> node (i, j+s, k+t); components (x, y, z)
  double vx = 0.0;
  if (i > 0) {
    for (int q = 0; q < 4; q++) disp(f, nidx(m, i, j + (q & 1), k + (q >> 1)), dt, g[q]);
    for (int q = 0; q < 4; q++) { d[q][0] = g[q][0]; d[q][1] = g[q][1]; d[q][2] = g[q][2]; }
    vx = swept_volume(d[0], d[1], d[2], d[3], m.dy, m.dz);
  }
  // y face at node plane j: corner (s,t) -> node (i+t, j, k+s); components (y, z, x)
  double vy = 0.0;
  if (j > 0) {
    for (int q = 0; q < 4; q++) disp(f, nidx(m, i + (q >> 1), j, k + (q & 1)), dt, g[q]);
    for (int q = 0; q < 4; q++) { d[q][0] = g[q][1]; d[q][1] = g[q][2]; d[q][2] = g[q][0]; }
    vy = swept_volume(d[0], d[1], d[2], d[3], m.dz, m.dx);
  }
  // z face at node plane k: corner (s,t) -> node (i+s, j+t, k); components (z, x, y)
  double vz = 0.0;
  if (k > 0) {
    for (int q = 0; q < 4; q++) disp(f, nidx(m, i + (q & 1), j + (q >> 1), k), dt, g[q]);
    for (int q = 0; q < 4; q++) { d[q][0] = g[q][2]; d[q][1] = g[q][0]; d[q][2] = g[q][1]; }
    vz = swept_volume(d[0], d[1], d[2], d[3], m.dx, m.dy);
  }
  f.dvx[c] = vx;
  f.dvy[c] = vy;
  f.dvz[c] = vz;
}

__global__ __launch_bounds__(TPB) void k_lagr(Mesh m, Ctl *ctl, Fields64 f) {
  if (ctl->done) return;
  const int64_t c = blockIdx.x * (int64_t)TPB + threadIdx.x;
  if (c >= m.ncell) return;
  int i, j, k;
  cell_ijk(m, c, i, j, k);
  const double dt = ctl->dt;
  const double mc = f.rho[c] * m.V0;
  const double work = corner_sum(m, i, j, k, [&](int a, int64_t n) {
    return a == 0 ? 0.5 * (f.u[n] + f.u1[n]) : (a == 1 ? 0.5 * (f.v[n] + f.v1[n]) : 0.5 * (f.w[n] + f.w1[n]));
  });
  f.eL[c] = f.e[c] - (dt / mc) * f.ps[c] * work;
  const double ux = (i + 1 < m.nx) ? f.dvx[c + 1] : 0.0;
  const double uy = (j + 1 < m.ny) ? f.dvy[c + m.nx] : 0.0;
  const double uz = (k + 1 < m.nz) ? f.dvz[c + (int64_t)m.nx * m.ny] : 0.0;
  const double VL = m.V0 + ((ux - f.dvx[c]) + (uy - f.dvy[c]) + (uz - f.dvz[c]));
  if (!(VL > 0.0)) {
    atomicOr(&ctl->status, SALE_FLAG_TANGLE);
    f.rhoL[c] = 0.0;
    return;
  }
  f.rhoL[c] = mc / VL;
}

__global__ __launch_bounds__(TPB) void k_flux(Mesh m, Ctl *ctl, Fields64 f) {
  if (ctl->done) return;
  const int64_t c = blockIdx.x * (int64_t)TPB + threadIdx.x;
  if (c >= m.ncell) return;
  int i, j, k;
  cell_ijk(m, c, i, j, k);
  const int64_t sy = m.nx, sz = (int64_t)m.nx * m.ny;
  double mu = 0.0, ep = 0.0;
  if (i > 0) {
    const double dv = f.dvx[c];
    const int64_t dn = dv > 0.0 ? c - 1 : c;
    mu = f.rhoL[dn] * dv;
    ep = mu * f.eL[dn];
  }
  f.mux[c] = mu;
  f.ex[c] = ep;
  mu = ep = 0.0;
  if (j > 0) {
    const double dv = f.dvy[c];
    const int64_t dn = dv > 0.0 ? c - sy : c;
    mu = f.rhoL[dn] * dv;
    ep = mu * f.eL[dn];
  }
  f.muy[c] = mu;
  f.ey[c] = ep;
  mu = ep = 0.0;
  if (k > 0) {
    const double dv = f.dvz[c];
    const int64_t dn = dv > 0.0 ? c - sz : c;
    mu = f.rhoL[dn] * dv;
    ep = mu * f.eL[dn];
  }
  f.muz[c] = mu;
  f.ez[c] = ep;
}

__global__ __launch_bounds__(TPB) void k_remap(Mesh m, Ctl *ctl, Fields64 f) {
  if (ctl->done) return;
  const int64_t c = blockIdx.x * (int64_t)TPB + threadIdx.x;
  if (c >= m.ncell) return;
  int i, j, k;
  cell_ijk(m, c, i, j, k);
  const int64_t sy = m.nx, sz = (int64_t)m.nx * m.ny;
  const bool hx = i + 1 < m.nx, hy = j + 1 < m.ny, hz = k + 1 < m.nz;
  const double netm = ((hx ? f.mux[c + 1] : 0.0) - f.mux[c]) + ((hy ? f.muy[c + sy] : 0.0) - f.muy[c]) +
                      ((hz ? f.muz[c + sz] : 0.0) - f.muz[c]);
  const double nete = ((hx ? f.ex[c + 1] : 0.0) - f.ex[c]) + ((hy ? f.ey[c + sy] : 0.0) - f.ey[c]) +
                      ((hz ? f.ez[c + sz] : 0.0) - f.ez[c]);
  const double rho = f.rho[c];
  const double mc = rho * m.V0;
  const double M = mc - netm;
  const double rn = rho - netm / m.V0;
  f.M[c] = M;
  f.rn[c] = rn;
  if (!(M > 0.0) || !(rn > 0.0)) {
    atomicOr(&ctl->status, SALE_FLAG_NUMERIC);
    f.epre[c] = 0.0;
    return;
  }
  const double eL = f.eL[c];
  f.epre[c] = eL + (eL * netm - nete) / M;
}

// dual-face mass flux between node (i,j,k) and its +axis neighbour
__device__ __forceinline__ double dual_flux(const Mesh &m, const Fields64 &f, int axis, int i, int j,
                                            int k) {
  double s = 0.0;
  for (int o2 = -1; o2 <= 0; o2++)
    for (int o1 = -1; o1 <= 0; o1++) {
      int ci = i, cj = j, ck = k;
      if (axis == 0) { cj += o1; ck += o2; }
      if (axis == 1) { ci += o1; ck += o2; }
      if (axis == 2) { ci += o1; cj += o2; }
      if (!cell_in(m, ci, cj, ck)) continue;
      const int64_t c = cidx(m, ci, cj, ck);
      if (axis == 0) s += f.mux[c] + (ci + 1 < m.nx ? f.mux[c + 1] : 0.0);
      if (axis == 1) s += f.muy[c] + (cj + 1 < m.ny ? f.muy[c + m.nx] : 0.0);
      if (axis == 2) s += f.muz[c] + (ck + 1 < m.nz ? f.muz[c + (int64_t)m.nx * m.ny] : 0.0);
    }
  return 0.125 * s;
}

__global__ __launch_bounds__(TPB) void k_node_remap(Mesh m, Ctl *ctl, Fields64 f) {
  if (ctl->done) return;
  const int64_t n = blockIdx.x * (int64_t)TPB + threadIdx.x;
  if (n >= m.nnode) return;
  int i, j, k;
  node_ijk(m, n, i, j, k);
  double sm = 0.0, sM = 0.0;
  for (int cc = -1; cc <= 0; cc++)
    for (int b = -1; b <= 0; b++)
      for (int a = -1; a <= 0; a++)
        if (cell_in(m, i + a, j + b, k + cc)) {
          const int64_t c = cidx(m, i + a, j + b, k + cc);
          sm += f.rho[c] * m.V0;
          sM += f.M[c];
        }
  const double mp = 0.125 * sm;
  const double mn = 0.125 * sM;
  const double u1 = f.u1[n], v1 = f.v1[n], w1 = f.w1[n];
  double P0 = mp * u1, P1 = mp * v1, P2 = mp * w1;
  double K = 0.5 * mp * (u1 * u1 + v1 * v1 + w1 * w1);
  const int lim[3] = {m.nx, m.ny, m.nz};
  const int idx[3] = {i, j, k};
  const int64_t st[3] = {1, m.nx + 1, (int64_t)(m.nx + 1) * (m.ny + 1)};
  for (int axis = 0; axis < 3; axis++) {
    if (idx[axis] + 1 <= lim[axis]) {  // edge to the +axis neighbour: outflow
      const double phi = dual_flux(m, f, axis, i, j, k);
      const int64_t dn = phi > 0.0 ? n : n + st[axis];
      const double ud = f.u1[dn], vd = f.v1[dn], wd = f.w1[dn];
      P0 -= phi * ud;
      P1 -= phi * vd;
      P2 -= phi * wd;
      K -= phi * 0.5 * (ud * ud + vd * vd + wd * wd);
    }
    if (idx[axis] - 1 >= 0) {  // edge from the -axis neighbour: inflow
      const double phi = dual_flux(m, f, axis, i - (axis == 0), j - (axis == 1), k - (axis == 2));
      const int64_t dn = phi > 0.0 ? n - st[axis] : n;
      const double ud = f.u1[dn], vd = f.v1[dn], wd = f.w1[dn];
      P0 += phi * ud;
      P1 += phi * vd;
      P2 += phi * wd;
      K += phi * 0.5 * (ud * ud + vd * vd + wd * wd);
    }
  }
  if (!(mn > 0.0)) {
    atomicOr(&ctl->status, SALE_FLAG_NUMERIC);
    f.u[n] = f.v[n] = f.w[n] = 0.0;
    f.dkm[n] = 0.0;
    return;
  }
  double un = P0 / mn, vn = P1 / mn, wn = P2 / mn;
  if (i == 0 || i == m.nx) un = 0.0;
  if (j == 0 || j == m.ny) vn = 0.0;
  if (k == 0 || k == m.nz) wn = 0.0;
  f.u[n] = un;  // u is not read again in this step: update in place
  f.v[n] = vn;
  f.w[n] = wn;
  f.dkm[n] = (K - 0.5 * mn * (un * un + vn * vn + wn * wn)) / mn;
}

__global__ __launch_bounds__(TPB) void k_finish(Mesh m, Ctl *ctl, Fields64 f) {
  if (ctl->done) return;
  const int64_t c = blockIdx.x * (int64_t)TPB + threadIdx.x;
  double a = 0.0;
  bool bad = false;
  if (c < m.ncell) {
    int i, j, k;
    cell_ijk(m, c, i, j, k);
    double s = 0.0;
#pragma unroll
    for (int cc = 0; cc < 2; cc++)
#pragma unroll
      for (int b = 0; b < 2; b++)
#pragma unroll
        for (int aa = 0; aa < 2; aa++) s += f.dkm[nidx(m, i + aa, j + b, k + cc)];
    const double en = f.epre[c] + 0.125 * s;
    const double rn = f.rn[c];
    f.e[c] = en;
    f.rho[c] = rn;
    a = signal_speed(m, i, j, k, rn, en, f.u, f.v, f.w, bad);
  }
  block_max_to_ctl(ctl, a, bad);
}

// signal speed of the current state (after init)
__global__ __launch_bounds__(TPB) void k_signal(Mesh m, Ctl *ctl, Fields64 f) {
  const int64_t c = blockIdx.x * (int64_t)TPB + threadIdx.x;
  double a = 0.0;
  bool bad = false;
  if (c < m.ncell) {
    int i, j, k;
    cell_ijk(m, c, i, j, k);
    a = signal_speed(m, i, j, k, f.rho[c], f.e[c], f.u, f.v, f.w, bad);
  }
  block_max_to_ctl(ctl, a, bad);
}

// ---- initial states -------------------------------------------------------------
__global__ void k_ctl_init(Ctl *ctl, double t0, long long step0, double t_end) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  ctl->t = t0;
  ctl->dt = 0.0;
  ctl->t_end = t_end;
  ctl->dt_next = 0.0;
  ctl->amax_bits = 0ull;
  ctl->step = step0;
  ctl->status = 0u;
  ctl->done = 0u;
  ctl->totals[0] = ctl->totals[1] = 0.0;
}

__global__ void k_set_t_end(Ctl *ctl, double t_end) {
  if (threadIdx.x == 0 && blockIdx.x == 0) ctl->t_end = t_end;
}

__global__ __launch_bounds__(TPB) void k_init_cells_sod(Mesh m, Fields64 f, double xs, double rL,
                                                       double pL, double rR, double pR, double lox) {
  const int64_t c = blockIdx.x * (int64_t)TPB + threadIdx.x;
  if (c >= m.ncell) return;
  int i, j, k;
  cell_ijk(m, c, i, j, k);
  const double xc = lox + (i + 0.5) * m.dx;
  const bool left = xc < xs;
  const double r = left ? rL : rR;
  f.rho[c] = r;
  f.e[c] = (left ? pL : pR) / ((m.gamma - 1.0) * r);
}

__global__ __launch_bounds__(TPB) void k_init_cells_sedov(Mesh m, Fields64 f, double r0, double p0,
                                                         double edep) {
  const int64_t c = blockIdx.x * (int64_t)TPB + threadIdx.x;
  if (c >= m.ncell) return;
  f.rho[c] = r0;
  f.e[c] = c == 0 ? edep / (r0 * m.V0) : p0 / ((m.gamma - 1.0) * r0);
}

__global__ __launch_bounds__(TPB) void k_zero_nodes(Mesh m, Fields64 f) {
  const int64_t n = blockIdx.x * (int64_t)TPB + threadIdx.x;
  if (n >= m.nnode) return;
  f.u[n] = f.v[n] = f.w[n] = 0.0;
}

__global__ __launch_bounds__(TPB) void k_wall_normals(Mesh m, Fields64 f) {
  const int64_t n = blockIdx.x * (int64_t)TPB + threadIdx.x;
  if (n >= m.nnode) return;
  int i, j, k;
  node_ijk(m, n, i, j, k);
  if (i == 0 || i == m.nx) f.u[n] = 0.0;
  if (j == 0 || j == m.ny) f.v[n] = 0.0;
  if (k == 0 || k == m.nz) f.w[n] = 0.0;
}

// ---- diagnostics: deterministic two-level sums ----------------------------------
constexpr int TOT_BLOCKS = 1024;

__global__ __launch_bounds__(TPB) void k_totals_partial(Mesh m, Fields64 f) {
  double sm = 0.0, si = 0.0, sk = 0.0;
  for (int64_t c = blockIdx.x * (int64_t)TPB + threadIdx.x; c < m.ncell; c += (int64_t)TOT_BLOCKS * TPB) {
    const double mc = f.rho[c] * m.V0;
    sm += mc;
    si += mc * f.e[c];
  }
  for (int64_t n = blockIdx.x * (int64_t)TPB + threadIdx.x; n < m.nnode; n += (int64_t)TOT_BLOCKS * TPB) {
    int i, j, k;
    node_ijk(m, n, i, j, k);
    double s = 0.0;
    for (int cc = -1; cc <= 0; cc++)
      for (int b = -1; b <= 0; b++)
        for (int a = -1; a <= 0; a++)
          if (cell_in(m, i + a, j + b, k + cc)) s += f.rho[cidx(m, i + a, j + b, k + cc)] * m.V0;
    sk += 0.5 * (0.125 * s) * (f.u[n] * f.u[n] + f.v[n] * f.v[n] + f.w[n] * f.w[n]);
  }
  __shared__ double red[3][TPB / 64];
  sm = wave_sum(sm);
  si = wave_sum(si);
  sk = wave_sum(sk);
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = sm;
    red[1][threadIdx.x >> 6] = si;
    red[2][threadIdx.x >> 6] = sk;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double r = 0.0;
    for (int q = 0; q < TPB / 64; q++) r += red[threadIdx.x][q];
    f.partial[threadIdx.x * TOT_BLOCKS + blockIdx.x] = r;
  }
}

__global__ __launch_bounds__(TPB) void k_totals_final(Ctl *ctl, Fields64 f) {
  __shared__ double red[3][TPB / 64];
  double s[3];
  for (int a = 0; a < 3; a++) {
    double x = 0.0;
    for (int b = threadIdx.x; b < TOT_BLOCKS; b += TPB) x += f.partial[a * TOT_BLOCKS + b];
    s[a] = wave_sum(x);
  }
  if ((threadIdx.x & 63) == 0)
    for (int a = 0; a < 3; a++) red[a][threadIdx.x >> 6] = s[a];
  __syncthreads();
  if (threadIdx.x == 0) {
    double r[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < 3; a++)
      for (int q = 0; q < TPB / 64; q++) r[a] += red[a][q];
    ctl->totals[0] = r[0];
    ctl->totals[1] = r[1] + r[2];
  }
}

__global__ __launch_bounds__(TPB) void k_derived(Mesh m, Fields64 f, int which, double *out) {
  const int64_t c = blockIdx.x * (int64_t)TPB + threadIdx.x;
  if (c >= m.ncell) return;
  const double rho = f.rho[c], e = f.e[c];
  if (which == 0) {
    out[c] = (m.gamma - 1.0) * rho * e;
    return;
  }
  int i, j, k;
  cell_ijk(m, c, i, j, k);
  const double cs = sqrt(m.gamma * (m.gamma - 1.0) * fmax(e, 0.0));
  const double D = corner_sum(m, i, j, k, [&](int a, int64_t n) {
                     return a == 0 ? f.u[n] : (a == 1 ? f.v[n] : f.w[n]);
                   }) / m.V0;
  double q = 0.0;
  if (D < 0.0) {
    const double hd = m.h * D;
    q = rho * (m.cq * hd * hd + m.cl * cs * m.h * fabs(D));
  }
  out[c] = q;
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + TPB - 1) / TPB); }

}  // namespace

// ---- workspace layout -------------------------------------------------------------
static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t workspace_bytes_fp64(const Mesh &m, size_t *ctl_off) {
  const size_t cb = align256((size_t)m.ncell * sizeof(double));
  const size_t nb = align256((size_t)m.nnode * sizeof(double));
  if (ctl_off) *ctl_off = 0;
  // ctl | 2 state cells + 3 state nodes | 16 cell temporaries | 4 node temporaries | partials
  return align256(sizeof(Ctl)) + 2 * cb + 3 * nb + 16 * cb + 4 * nb +
         align256(3 * TOT_BLOCKS * sizeof(double));
}

void layout_fp64(const Mesh &m, void *ws, Ctl **ctl, Fields64 *f) {
  const size_t cb = align256((size_t)m.ncell * sizeof(double));
  const size_t nb = align256((size_t)m.nnode * sizeof(double));
  char *p = (char *)ws;
  *ctl = (Ctl *)p;
  p += align256(sizeof(Ctl));
  auto take = [&](size_t b) { double *r = (double *)p; p += b; return r; };
  f->rho = take(cb); f->e = take(cb);
  f->u = take(nb); f->v = take(nb); f->w = take(nb);
  f->ps = take(cb); f->rhoL = take(cb); f->eL = take(cb);
  f->dvx = take(cb); f->dvy = take(cb); f->dvz = take(cb);
  f->mux = take(cb); f->muy = take(cb); f->muz = take(cb);
  f->ex = take(cb); f->ey = take(cb); f->ez = take(cb);
  f->M = take(cb); f->rn = take(cb); f->epre = take(cb);
  f->scratch = take(cb);
  f->u1 = take(nb); f->v1 = take(nb); f->w1 = take(nb); f->dkm = take(nb);
  f->partial = take(align256(3 * TOT_BLOCKS * sizeof(double)));
  f->npartial = 3 * TOT_BLOCKS;
}

// ---- launchers ------------------------------------------------------------------------
static hipError_t finish_init(const Mesh &m, Ctl *ctl, const Fields64 &f, double t0, long long step0,
                              double t_end, hipStream_t s) {
  hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, s, ctl, t0, step0, t_end);
  hipLaunchKernelGGL(k_signal, dim3(blocks(m.ncell)), dim3(TPB), 0, s, m, ctl, f);
  return hipGetLastError();
}

hipError_t launch_init_sod(const Mesh &m, Ctl *ctl, const Fields64 &f, const double sod[5], double t0,
                           long long step0, double t_end, hipStream_t s) {
  hipLaunchKernelGGL(k_init_cells_sod, dim3(blocks(m.ncell)), dim3(TPB), 0, s, m, f, sod[0], sod[1],
                     sod[2], sod[3], sod[4], m.lo[0]);
  hipLaunchKernelGGL(k_zero_nodes, dim3(blocks(m.nnode)), dim3(TPB), 0, s, m, f);
  return finish_init(m, ctl, f, t0, step0, t_end, s);
}

hipError_t launch_init_sedov(const Mesh &m, Ctl *ctl, const Fields64 &f, const double sedov[3],
                             double t0, long long step0, double t_end, hipStream_t s) {
  hipLaunchKernelGGL(k_init_cells_sedov, dim3(blocks(m.ncell)), dim3(TPB), 0, s, m, f, sedov[0],
                     sedov[1], sedov[2]);
  hipLaunchKernelGGL(k_zero_nodes, dim3(blocks(m.nnode)), dim3(TPB), 0, s, m, f);
  return finish_init(m, ctl, f, t0, step0, t_end, s);
}

hipError_t launch_init_user(const Mesh &m, Ctl *ctl, const Fields64 &f, double t0, long long step0,
                            double t_end, hipStream_t s) {
  hipLaunchKernelGGL(k_wall_normals, dim3(blocks(m.nnode)), dim3(TPB), 0, s, m, f);
  return finish_init(m, ctl, f, t0, step0, t_end, s);
}

hipError_t launch_set_t_end(Ctl *ctl, double t_end, hipStream_t s) {
  hipLaunchKernelGGL(k_set_t_end, dim3(1), dim3(64), 0, s, ctl, t_end);
  return hipGetLastError();
}

hipError_t launch_step_fp64(const Mesh &m, Ctl *ctl, const Fields64 &f, hipStream_t s) {
  const unsigned bc = blocks(m.ncell), bn = blocks(m.nnode);
  hipLaunchKernelGGL(k_begin, dim3(1), dim3(64), 0, s, m, ctl);
  hipLaunchKernelGGL(k_predict, dim3(bc), dim3(TPB), 0, s, m, ctl, f);
  hipLaunchKernelGGL(k_accel, dim3(bn), dim3(TPB), 0, s, m, ctl, f);
  hipLaunchKernelGGL(k_swept, dim3(bc), dim3(TPB), 0, s, m, ctl, f);
  hipLaunchKernelGGL(k_lagr, dim3(bc), dim3(TPB), 0, s, m, ctl, f);
  hipLaunchKernelGGL(k_flux, dim3(bc), dim3(TPB), 0, s, m, ctl, f);
  hipLaunchKernelGGL(k_remap, dim3(bc), dim3(TPB), 0, s, m, ctl, f);
  hipLaunchKernelGGL(k_node_remap, dim3(bn), dim3(TPB), 0, s, m, ctl, f);
  hipLaunchKernelGGL(k_finish, dim3(bc), dim3(TPB), 0, s, m, ctl, f);
  return hipGetLastError();
}

hipError_t launch_totals_fp64(const Mesh &m, Ctl *ctl, const Fields64 &f, hipStream_t s) {
  hipLaunchKernelGGL(k_totals_partial, dim3(TOT_BLOCKS), dim3(TPB), 0, s, m, f);
  hipLaunchKernelGGL(k_totals_final, dim3(1), dim3(TPB), 0, s, ctl, f);
  return hipGetLastError();
}

hipError_t launch_derived_fp64(const Mesh &m, const Fields64 &f, int which, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_derived, dim3(blocks(m.ncell)), dim3(TPB), 0, s, m, f, which, out);
  return hipGetLastError();
}

}  // namespace sale
