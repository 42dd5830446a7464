// sale_remap2.hip -- the second-order remap of libsale (gfx950): the
// Eulerian rezone and advection (ScalSALE Sec. I-D and Table I) with donor
// values taken from limited linear profiles instead of the donor's mean.
//
// Reading (the paper leaves the advection's order open): along each face
// normal, the donor cell's rho^L and e^L (and, on the dual mesh, the donor
// node's u') are replaced by the value of a linear profile at the centroid
// of the swept slab, |dv| / area thick, at the donor's end next to the face;
// the profile's slope is the harmonic (van Leer) mean of the one-sided
// differences, zero where they differ in sign or where the neighbour along
// that axis is a wall. The dual face's swept volume is the 1/8 average of the
// adjacent cells' face swept volumes, like its mass flux. Everything else --
// masses, the dual fluxes, the kinetic-energy fix, walls, the next signal
// speed -- is the first-order step's.
//
// Four passes, one thread per cell or node, neighbours read through the
// caches (a direct form; the first-order remap is the tiled one):
//   k_faces2  fluxes through each cell's three lower faces
//   k_cells2  M, rho^{n+1}, e^pre
//   k_nodes2  dual fluxes, reconstructed donor velocities, u^{n+1}, KE defect
//   k_fix2    KE fix, e^{n+1}, the next signal speed (block max -> ctl)
// A step after t_end or after an error flag copies the state instead.
#include "sale_tiles.h"

namespace sale {
namespace {

constexpr int TPB2 = 256;

inline int64_t blocks2(int64_t n) { return (n + TPB2 - 1) / TPB2; }

template <typename R>
__device__ __forceinline__ R vanleer(R am, R ap) {
  return (am * ap > R(0)) ? R(2) * am * ap / (am + ap) : R(0);
}

// value of the donor's profile (mean q, slope) at the centroid of the swept
// slab; dvA = swept volume / face area, > 0 when the donor is the lower cell
template <typename R>
__device__ __forceinline__ R donor_value(R q, R slope, R h, R dvA) {
  const R off = R(0.5) * (h - fabs(dvA));
  return dvA > R(0) ? q + slope * off : q - slope * off;
}

__device__ __forceinline__ void cell_of(const Mesh &m, int64_t c, int &i, int &j, int &k) {
  i = (int)(c % m.nx);
  const int64_t r = c / m.nx;
  j = (int)(r % m.ny);
  k = (int)(r / m.ny);
}
__device__ __forceinline__ void node_of(const Mesh &m, int64_t n, int &i, int &j, int &k) {
  i = (int)(n % (m.nx + 1));
  const int64_t r = n / (m.nx + 1);
  j = (int)(r % (m.ny + 1));
  k = (int)(r / (m.ny + 1));
}

// ---- pass 1: face fluxes ---------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(TPB2) void k_faces2(Mesh m, const Ctl *ctl, Geo<R> geo, Rem2<R> t) {
  const int64_t c = blockIdx.x * (int64_t)TPB2 + threadIdx.x;
  if (c >= m.ncell || ctl->done) return;
  int idx[3];
  cell_of(m, c, idx[0], idx[1], idx[2]);
  const int n3[3] = {m.nx, m.ny, m.nz};
  const int64_t st[3] = {1, m.nx, (int64_t)m.nx * m.ny};
  const R *dvs[3] = {geo.dvx, geo.dvy, geo.dvz};
  const R hs[3] = {R(m.dx), R(m.dy), R(m.dz)};
  const R area[3] = {R(m.hyz), R(m.hzx), R(m.hxy)};
#pragma unroll
  for (int a = 0; a < 3; a++) {
    R mu = R(0), eps = R(0);
    if (idx[a] > 0) {  // interior lower face between c - e_a and c
      const R dv = dvs[a][c];
      const bool lower = dv > R(0);
      const int64_t dn = lower ? c - st[a] : c;
      const int di = lower ? idx[a] - 1 : idx[a];
      R sr = R(0), se = R(0);
      if (di >= 1 && di + 1 < n3[a]) {
        const R r0 = geo.rl[dn], rm = geo.rl[dn - st[a]], rp = geo.rl[dn + st[a]];
        const R e0 = geo.el[dn], em = geo.el[dn - st[a]], ep = geo.el[dn + st[a]];
        sr = vanleer((r0 - rm) / hs[a], (rp - r0) / hs[a]);
        se = vanleer((e0 - em) / hs[a], (ep - e0) / hs[a]);
      }
      const R dvA = dv / area[a];
      const R rf = donor_value(geo.rl[dn], sr, hs[a], dvA);
      const R ef = donor_value(geo.el[dn], se, hs[a], dvA);
      mu = rf * dv;
      eps = mu * ef;
    }
    t.mu[a][c] = mu;
    t.eps[a][c] = eps;
  }
}

// ---- pass 2: cell masses, densities, pre-fix energies ---------------------------------
template <typename R>
__global__ __launch_bounds__(TPB2) void k_cells2(Mesh m, Ctl *ctl, State<R> cur, State<R> nxt, Geo<R> geo,
                                                 Rem2<R> t) {
  const int64_t c = blockIdx.x * (int64_t)TPB2 + threadIdx.x;
  if (c >= m.ncell) return;
  if (ctl->done) {
    nxt.rho[c] = cur.rho[c];
    return;
  }
  int i, j, k;
  cell_of(m, c, i, j, k);
  const R zero = R(0);
  // upper faces are the +axis neighbours' lower faces, or walls
  const R mxu = i + 1 < m.nx ? t.mu[0][c + 1] : zero, exu = i + 1 < m.nx ? t.eps[0][c + 1] : zero;
  const R myu = j + 1 < m.ny ? t.mu[1][c + m.nx] : zero, eyu = j + 1 < m.ny ? t.eps[1][c + m.nx] : zero;
  const int64_t pz = (int64_t)m.nx * m.ny;
  const R mzu = k + 1 < m.nz ? t.mu[2][c + pz] : zero, ezu = k + 1 < m.nz ? t.eps[2][c + pz] : zero;
  const R netm = ((mxu - t.mu[0][c]) + (myu - t.mu[1][c])) + (mzu - t.mu[2][c]);
  const R nete = ((exu - t.eps[0][c]) + (eyu - t.eps[1][c])) + (ezu - t.eps[2][c]);
  const R rho = cur.rho[c];
  const R M = rho * R(m.V0) - netm;
  const R rn = rho - netm * R(m.iV0);
  R ep = R(0);
  if (!(M > R(0)) || !(rn > R(0)) || !isfinite(rn)) {
    atomicOr(&ctl->status, SALE_FLAG_NUMERIC);
  } else {
    const R el = geo.el[c];
    ep = el + (el * netm - nete) / M;
  }
  nxt.rho[c] = rn;
  t.M[c] = M;
  t.epre[c] = ep;
}

// ---- pass 3: node momentum and kinetic-energy remap ------------------------------------
template <typename R>
__global__ __launch_bounds__(TPB2) void k_nodes2(Mesh m, Ctl *ctl, State<R> cur, State<R> nxt, Geo<R> geo,
                                                 const R *up, const R *vp, const R *wp, Rem2<R> t) {
  const int64_t n = blockIdx.x * (int64_t)TPB2 + threadIdx.x;
  if (n >= m.nnode) return;
  if (ctl->done) {
    nxt.u[n] = cur.u[n];
    nxt.v[n] = cur.v[n];
    nxt.w[n] = cur.w[n];
    return;
  }
  int idx[3];
  node_of(m, n, idx[0], idx[1], idx[2]);
  const int i = idx[0], j = idx[1], k = idx[2];
  const int n3[3] = {m.nx, m.ny, m.nz};
  const int64_t cst[3] = {1, m.nx, (int64_t)m.nx * m.ny};
  const int64_t nst[3] = {1, m.nx + 1, (int64_t)(m.nx + 1) * (m.ny + 1)};
  const R *dvs[3] = {geo.dvx, geo.dvy, geo.dvz};
  const R hs[3] = {R(m.dx), R(m.dy), R(m.dz)};
  const R area[3] = {R(m.hyz), R(m.hzx), R(m.hxy)};
  const R *vel[3] = {up, vp, wp};
  // nodal mass of the old state and of the new one
  R m_old = R(0), m_new = R(0);
  for (int cc = -1; cc <= 0; cc++)
    for (int b = -1; b <= 0; b++)
      for (int a = -1; a <= 0; a++)
        if (cell_in(m, i + a, j + b, k + cc)) {
          const int64_t c = cidx(m, i + a, j + b, k + cc);
          m_old += cur.rho[c] * R(m.V0);
          m_new += t.M[c];
        }
  const R mp = R(0.125) * m_old, mn = R(0.125) * m_new;
  const R u1 = up[n], v1 = vp[n], w1 = wp[n];
  R P[3] = {mp * u1, mp * v1, mp * w1};
  R K = R(0.5) * mp * (u1 * u1 + v1 * v1 + w1 * w1);
  // mass flux and swept volume of the dual face of the edge from node
  // (i,j,k) + (lo along axis a) to its +a neighbour: 1/8 of the lower plus
  // upper face values of the (up to 4) cells sharing that edge
  auto dual = [&](int a, int e0, R &phi, R &dv) {
    R sp = R(0), sv = R(0);
    const int t1 = (a + 1) % 3, t2 = (a + 2) % 3;
    for (int o2 = -1; o2 <= 0; o2++)
      for (int o1 = -1; o1 <= 0; o1++) {
        int ci[3] = {i, j, k};
        ci[a] = e0;
        ci[t1] += o1;
        ci[t2] += o2;
        if (!cell_in(m, ci[0], ci[1], ci[2])) continue;
        const int64_t c = cidx(m, ci[0], ci[1], ci[2]);
        const bool up_in = ci[a] + 1 < n3[a];
        sp += t.mu[a][c] + (up_in ? t.mu[a][c + cst[a]] : R(0));
        sv += dvs[a][c] + (up_in ? dvs[a][c + cst[a]] : R(0));
      }
    phi = R(0.125) * sp;
    dv = R(0.125) * sv;
  };
  // donor velocity of an edge: the donor node's limited linear profile along
  // the edge at the dual swept slab's centroid
  auto donor = [&](int a, int64_t nlo, int ilo, R phi, R dv, R ud[3]) {
    const bool lower = phi > R(0);
    const int64_t dn = lower ? nlo : nlo + nst[a];
    const int di = lower ? ilo : ilo + 1;
    const R dvA = lower ? fabs(dv / area[a]) : -fabs(dv / area[a]);
    const bool both = di >= 1 && di + 1 <= n3[a];
#pragma unroll
    for (int q = 0; q < 3; q++) {
      const R v0 = vel[q][dn];
      R sl = R(0);
      if (both) sl = vanleer((v0 - vel[q][dn - nst[a]]) / hs[a], (vel[q][dn + nst[a]] - v0) / hs[a]);
      ud[q] = both ? donor_value(v0, sl, hs[a], dvA) : v0;
    }
  };
  auto flow = [&](R phi, const R ud[3], R sgn) {
    P[0] += sgn * (phi * ud[0]);
    P[1] += sgn * (phi * ud[1]);
    P[2] += sgn * (phi * ud[2]);
    K += sgn * (phi * R(0.5) * (ud[0] * ud[0] + ud[1] * ud[1] + ud[2] * ud[2]));
  };
  for (int a = 0; a < 3; a++) {
    if (idx[a] + 1 <= n3[a]) {  // edge to the +a neighbour: outflow
      R phi, dv, ud[3];
      dual(a, idx[a], phi, dv);
      donor(a, n, idx[a], phi, dv, ud);
      flow(phi, ud, R(-1));
    }
    if (idx[a] - 1 >= 0) {  // edge from the -a neighbour: inflow
      R phi, dv, ud[3];
      dual(a, idx[a] - 1, phi, dv);
      donor(a, n - nst[a], idx[a] - 1, phi, dv, ud);
      flow(phi, ud, R(1));
    }
  }
  R un = R(0), vn = R(0), wn = R(0), dk = R(0);
  if (!(mn > R(0))) {
    atomicOr(&ctl->status, SALE_FLAG_NUMERIC);
  } else {
    const R imn = R(1) / mn;
    un = P[0] * imn;
    vn = P[1] * imn;
    wn = P[2] * imn;
    if (i == 0 || i == m.nx) un = R(0);
    if (j == 0 || j == m.ny) vn = R(0);
    if (k == 0 || k == m.nz) wn = R(0);
    dk = (K - R(0.5) * mn * (un * un + vn * vn + wn * wn)) * imn;
  }
  nxt.u[n] = un;
  nxt.v[n] = vn;
  nxt.w[n] = wn;
  t.dk[n] = dk;
}

// ---- pass 4: kinetic-energy fix, new energy, next signal speed ------------------------
template <typename R>
__global__ __launch_bounds__(TPB2) void k_fix2(Mesh m, Ctl *ctl, State<R> cur, State<R> nxt, Rem2<R> t) {
  const int64_t c = blockIdx.x * (int64_t)TPB2 + threadIdx.x;
  const bool done = ctl->done;
  double a = 0.0;
  bool bad = false;
  if (c < m.ncell) {
    if (done) {
      nxt.e[c] = cur.e[c];
    } else {
      int i, j, k;
      cell_of(m, c, i, j, k);
      // the cell's 8 nodes, loaded once: KE defects, speeds, divergence
      R uu[2][2][2], vv[2][2][2], ww[2][2][2];
      R s = R(0), smax = R(0);
      for (int cc = 0; cc < 2; cc++)
        for (int b = 0; b < 2; b++)
          for (int aa = 0; aa < 2; aa++) {
            const int64_t nn = nidx(m, i + aa, j + b, k + cc);
            s += t.dk[nn];
            uu[cc][b][aa] = nxt.u[nn];
            vv[cc][b][aa] = nxt.v[nn];
            ww[cc][b][aa] = nxt.w[nn];
            smax = fmax(smax, speed(uu[cc][b][aa], vv[cc][b][aa], ww[cc][b][aa]));
          }
      const R en = t.epre[c] + R(0.125) * s;
      nxt.e[c] = en;
      // D as state_divergence forms it (same halves, same order)
      R xh[2], yh[2], zh[2];
      for (int cc = 0; cc < 2; cc++) {
        xh[cc] = (uu[cc][0][1] - uu[cc][0][0]) + (uu[cc][1][1] - uu[cc][1][0]);
        yh[cc] = (vv[cc][1][0] - vv[cc][0][0]) + (vv[cc][1][1] - vv[cc][0][1]);
        zh[cc] = ((ww[cc][0][0] + ww[cc][0][1]) + ww[cc][1][0]) + ww[cc][1][1];
      }
      const R D = divergence(m, xh[0], xh[1], yh[0], yh[1], zh[0], zh[1]);
      const R sa = signal_from(m, D, en, smax);
      if (!(en >= R(0)) || !isfinite(en) || !isfinite(sa))
        bad = true;
      else
        a = (double)sa;
    }
  }
  if (done) return;  // uniform: every thread of the launch sees the same flag
  block_max_to_ctl<TPB2>(ctl, a, bad);
}

}  // namespace

template <typename R>
hipError_t launch_remap2(const Mesh &m, Ctl *ctl, const Work<R> &w, int cur, hipStream_t s) {
  if (m.order != 2 || !w.r2.M) return hipErrorInvalidValue;
  const State<R> sc = w.s[cur], sn = w.s[1 - cur];
  const dim3 gc((unsigned)blocks2(m.ncell)), gn((unsigned)blocks2(m.nnode)), b(TPB2);
  hipLaunchKernelGGL(k_faces2<R>, gc, b, 0, s, m, ctl, w.geo, w.r2);
  hipLaunchKernelGGL(k_cells2<R>, gc, b, 0, s, m, ctl, sc, sn, w.geo, w.r2);
  hipLaunchKernelGGL(k_nodes2<R>, gn, b, 0, s, m, ctl, sc, sn, w.geo, w.up, w.vp, w.wp, w.r2);
  hipLaunchKernelGGL(k_fix2<R>, gc, b, 0, s, m, ctl, sc, sn, w.r2);
  return hipGetLastError();
}

template hipError_t launch_remap2<double>(const Mesh &, Ctl *, const Work<double> &, int, hipStream_t);
template hipError_t launch_remap2<float>(const Mesh &, Ctl *, const Work<float> &, int, hipStream_t);

}  // namespace sale
