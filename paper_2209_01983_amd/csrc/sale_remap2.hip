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
// Four passes; the first three one thread per cell or node with neighbours
// read through the caches (a direct form; the first-order remap is tiled):
//   k_faces2  fluxes through each cell's three lower faces
//   k_cells2  M, rho^{n+1}, e^pre
//   k_nodes2  dual fluxes, reconstructed donor velocities, u^{n+1}, KE defect
//   k_fix2    KE fix, e^{n+1}, the next signal speed (block max -> ctl); a
//             z-marching tile, each node plane read once
// A step after t_end or after an error flag copies the state instead.
#include "sale_tiles.h"

namespace sale {
namespace {

constexpr int TPB2 = 256;

inline int64_t blocks2(int64_t n) { return (n + TPB2 - 1) / TPB2; }

// Harmonic mean of two one-sided differences of neighbouring means (zero
// where they differ in sign): the limited change of the profile over one
// cell. The slope is this over the spacing h; it is applied as the fraction
// (h - |dv/A|) / (2h) of it (donor_weight), so a face needs one division per
// field (the mean) instead of three.
template <typename R>
__device__ __forceinline__ R vanleer(R dm, R dp) {
  return (dm * dp > R(0)) ? R(2) * dm * dp / (dm + dp) : R(0);
}

// distance from the donor's centre to the swept slab's centroid, in units
// of the cell: (h - |dvA|) / (2h); dvA = swept volume / face area
template <typename R>
__device__ __forceinline__ R donor_weight(R dvA, R ih) {
  return R(0.5) - R(0.5) * (fabs(dvA) * ih);
}

// value of the donor's profile (mean q, limited change dq over one cell) at
// the slab's centroid, on the face side of the donor: toward +axis when the
// donor is the lower cell (lower = true)
template <typename R>
__device__ __forceinline__ R donor_value(R q, R dq, R wgt, bool lower) {
  return lower ? q + dq * wgt : q - dq * wgt;
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
  // 1 / (h A): the slab's thickness over the spacing is |dv| / (h A)
  const R ihA[3] = {R(1) / (R(m.dx) * R(m.hyz)), R(1) / (R(m.dy) * R(m.hzx)), R(1) / (R(m.dz) * R(m.hxy))};
#pragma unroll
  for (int a = 0; a < 3; a++) {
    R mu = R(0), eps = R(0);
    if (idx[a] > 0) {  // interior lower face between c - e_a and c
      const R dv = dvs[a][c];
      const bool lower = dv > R(0);
      const int64_t dn = lower ? c - st[a] : c;
      const int di = lower ? idx[a] - 1 : idx[a];
      const R r0 = geo.rl[dn], e0 = geo.el[dn];
      R rf = r0, ef = e0;
      if (di >= 1 && di + 1 < n3[a]) {
        const R rm = geo.rl[dn - st[a]], rp = geo.rl[dn + st[a]];
        const R em = geo.el[dn - st[a]], ep = geo.el[dn + st[a]];
        const R wgt = donor_weight(dv, ihA[a]);
        rf = donor_value(r0, vanleer(r0 - rm, rp - r0), wgt, lower);
        ef = donor_value(e0, vanleer(e0 - em, ep - e0), wgt, lower);
      }
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
  const R ihA[3] = {R(1) / (R(m.dx) * R(m.hyz)), R(1) / (R(m.dy) * R(m.hzx)), R(1) / (R(m.dz) * R(m.hxy))};
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
  // mass fluxes and swept volumes of the dual faces of the node's two edges
  // along axis a (to the -a and to the +a neighbour): 1/8 of the lower plus
  // upper face values of the (up to 4) cells sharing each edge. The cells of
  // a transverse column at a-index i-1 and i share the face at node plane
  // i, so each column reads three faces for both edges.
  auto duals = [&](int a, R &phi_in, R &dv_in, R &phi_out, R &dv_out) {
    const int t1 = (a + 1) % 3, t2 = (a + 2) % 3;
    const int ia = idx[a];
    const bool has_in = ia >= 1, has_out = ia + 1 <= n3[a];
    R spi = R(0), svi = R(0), spo = R(0), svo = R(0);
    for (int o2 = -1; o2 <= 0; o2++)
      for (int o1 = -1; o1 <= 0; o1++) {
        int ci[3] = {i, j, k};
        ci[t1] += o1;
        ci[t2] += o2;
        if (ci[t1] < 0 || ci[t1] >= n3[t1] || ci[t2] < 0 || ci[t2] >= n3[t2]) continue;
        ci[a] = 0;
        const int64_t c0 = cidx(m, ci[0], ci[1], ci[2]) + (int64_t)ia * cst[a];  // cell at a-index ia
        // faces at node planes ia - 1, ia, ia + 1 (zero on the walls)
        R mm = R(0), vm = R(0), m0 = R(0), v0 = R(0), mp = R(0), vp = R(0);
        if (has_in) {
          mm = t.mu[a][c0 - cst[a]];
          vm = dvs[a][c0 - cst[a]];
        }
        if (has_out) {
          m0 = t.mu[a][c0];
          v0 = dvs[a][c0];
          if (ia + 1 < n3[a]) {
            mp = t.mu[a][c0 + cst[a]];
            vp = dvs[a][c0 + cst[a]];
          }
          spo += m0 + mp;
          svo += v0 + vp;
        }
        if (has_in) {
          spi += mm + m0;
          svi += vm + v0;
        }
      }
    phi_in = R(0.125) * spi;
    dv_in = R(0.125) * svi;
    phi_out = R(0.125) * spo;
    dv_out = R(0.125) * svo;
  };
  // donor velocity of an edge: the donor node's limited linear profile along
  // the edge at the dual swept slab's centroid
  auto donor = [&](int a, int64_t nlo, int ilo, R phi, R dv, R ud[3]) {
    const bool lower = phi > R(0);
    const int64_t dn = lower ? nlo : nlo + nst[a];
    const int di = lower ? ilo : ilo + 1;
    const bool both = di >= 1 && di + 1 <= n3[a];
    const R wgt = donor_weight(dv, ihA[a]);
    // the slab lies on the +a side of the donor when the donor is the lower
    // node and the dual swept volume is not zero
    const bool plus = lower && dv != R(0);
#pragma unroll
    for (int q = 0; q < 3; q++) {
      const R v0 = vel[q][dn];
      ud[q] = both ? donor_value(v0, vanleer(v0 - vel[q][dn - nst[a]], vel[q][dn + nst[a]] - v0), wgt, plus) : v0;
    }
  };
  auto flow = [&](R phi, const R ud[3], R sgn) {
    P[0] += sgn * (phi * ud[0]);
    P[1] += sgn * (phi * ud[1]);
    P[2] += sgn * (phi * ud[2]);
    K += sgn * (phi * R(0.5) * (ud[0] * ud[0] + ud[1] * ud[1] + ud[2] * ud[2]));
  };
  for (int a = 0; a < 3; a++) {
    R phi_in, dv_in, phi_out, dv_out;
    duals(a, phi_in, dv_in, phi_out, dv_out);
    if (idx[a] + 1 <= n3[a]) {  // edge to the +a neighbour: outflow
      R ud[3];
      donor(a, n, idx[a], phi_out, dv_out, ud);
      flow(phi_out, ud, R(-1));
    }
    if (idx[a] - 1 >= 0) {  // edge from the -a neighbour: inflow
      R ud[3];
      donor(a, n - nst[a], idx[a] - 1, phi_in, dv_in, ud);
      flow(phi_in, ud, R(1));
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
// A 32 x 16 tile of node columns marched along z over one segment: each
// node plane's u^{n+1}, v, w and KE defect are read once into LDS, a cell
// column forms its lower-plane half (partial defect sum, largest |u|^2,
// divergence halves) and finishes the cell when the upper plane arrives.
// Sums run in the order of the cell's 8 nodes (x fastest, then y, then z),
// as in the gather form of the same pass.
constexpr int FW = 32, FH = 16, FTX = FW - 1, FTY = FH - 1;

template <typename R>
__global__ __launch_bounds__(FW * FH) void k_fix2(Mesh m, Ctl *ctl, State<R> cur, State<R> nxt, Rem2<R> t, Grid2 g) {
  __shared__ R sU[FH][FW], sV[FH][FW], sW[FH][FW], sQ[FH][FW];
  int tx, ty, seg;
  tile_of(g, blockIdx.x, tx, ty, seg);
  const int ci = threadIdx.x % FW, cj = threadIdx.x / FW;
  const int gi = tx * FTX + ci, gj = ty * FTY + cj;  // node column; cell column when owned
  const int Z0 = seg * g.seglen;
  const int Z1 = seg == g.nseg - 1 ? m.nz : Z0 + g.seglen;  // cell planes [Z0, Z1)
  const bool ncol = gi <= m.nx && gj <= m.ny;
  const bool own = ci < FTX && cj < FTY && gi < m.nx && gj < m.ny;
  const int64_t cpl = (int64_t)m.nx * m.ny, npl = (int64_t)(m.nx + 1) * (m.ny + 1);
  const int64_t cix = own ? gi + (int64_t)m.nx * gj : 0, nix = ncol ? gi + (int64_t)(m.nx + 1) * gj : 0;
  if (ctl->done) {  // uniform: the state is carried over
    if (own)
      for (int k = Z0; k < Z1; k++) nxt.e[cix + k * cpl] = cur.e[cix + k * cpl];
    return;
  }
  R fu = 0, fv = 0, fw = 0, fq = 0;  // node plane loads, one plane ahead
  auto fetch = [&](int k) {
    fu = fv = fw = fq = R(0);
    if (ncol && k <= m.nz) {
      const int64_t q = nix + k * npl;
      fu = nxt.u[q];
      fv = nxt.v[q];
      fw = nxt.w[q];
      fq = t.dk[q];
    }
  };
  fetch(Z0);
  R s_lo = 0, s2_lo = 0, xh_lo = 0, yh_lo = 0, zh_lo = 0;  // lower node plane of the cell
  double a = 0.0;
  bool bad = false;
  for (int k = Z0; k <= Z1; k++) {  // node plane k: upper plane of cell k-1, lower of cell k
    sU[cj][ci] = fu;
    sV[cj][ci] = fv;
    sW[cj][ci] = fw;
    sQ[cj][ci] = fq;
    fetch(k + 1);
    __syncthreads();
    if (own) {
      const R u00 = sU[cj][ci], u01 = sU[cj][ci + 1], u10 = sU[cj + 1][ci], u11 = sU[cj + 1][ci + 1];
      const R v00 = sV[cj][ci], v01 = sV[cj][ci + 1], v10 = sV[cj + 1][ci], v11 = sV[cj + 1][ci + 1];
      const R w00 = sW[cj][ci], w01 = sW[cj][ci + 1], w10 = sW[cj + 1][ci], w11 = sW[cj + 1][ci + 1];
      const R q00 = sQ[cj][ci], q01 = sQ[cj][ci + 1], q10 = sQ[cj + 1][ci], q11 = sQ[cj + 1][ci + 1];
      const R s2 = fmax(fmax(fma(w00, w00, fma(v00, v00, u00 * u00)), fma(w01, w01, fma(v01, v01, u01 * u01))),
                        fmax(fma(w10, w10, fma(v10, v10, u10 * u10)), fma(w11, w11, fma(v11, v11, u11 * u11))));
      const R xh = (u01 - u00) + (u11 - u10);
      const R yh = (v10 - v00) + (v11 - v01);
      const R zh = ((w00 + w01) + w10) + w11;
      if (k > Z0) {  // finish cell k-1
        const R s = (((s_lo + q00) + q01) + q10) + q11;
        const int64_t c = cix + (k - 1) * cpl;
        const R en = t.epre[c] + R(0.125) * s;
        nxt.e[c] = en;
        const R D = divergence(m, xh_lo, xh, yh_lo, yh, zh_lo, zh);
        // the square root is monotone: this is the largest speed() of the 8 nodes
        const R sa = signal_from(m, D, en, sqrt(fmax(s2_lo, s2)));
        if (!(en >= R(0)) || !isfinite(en) || !isfinite(sa))
          bad = true;
        else
          a = fmax(a, (double)sa);
      }
      s_lo = ((q00 + q01) + q10) + q11;
      s2_lo = s2;
      xh_lo = xh;
      yh_lo = yh;
      zh_lo = zh;
    }
    __syncthreads();
  }
  block_max_to_ctl<FW * FH>(ctl, a, bad);
}

}  // namespace

template <typename R>
hipError_t launch_remap2(const Mesh &m, Ctl *ctl, const Work<R> &w, int cur, hipStream_t s) {
  if (m.order != 2 || !w.r2.M) return hipErrorInvalidValue;
  const State<R> sc = w.s[cur], sn = w.s[1 - cur];
  const dim3 gc((unsigned)blocks2(m.ncell)), gn((unsigned)blocks2(m.nnode)), b(TPB2);
  // KE-fix tiles: about 3072 blocks, at least 8 cell planes per segment
  Grid2 gf;
  gf.tx = (m.nx + FTX - 1) / FTX;
  gf.ty = (m.ny + FTY - 1) / FTY;
  const int maxseg = m.nz / 8 > 1 ? m.nz / 8 : 1;
  int nseg = (3072 + gf.tx * gf.ty / 2) / (gf.tx * gf.ty);
  nseg = nseg < 1 ? 1 : nseg > maxseg ? maxseg : nseg;
  gf.seglen = (m.nz + nseg - 1) / nseg;
  gf.nseg = (m.nz + gf.seglen - 1) / gf.seglen;
  hipLaunchKernelGGL(k_faces2<R>, gc, b, 0, s, m, ctl, w.geo, w.r2);
  hipLaunchKernelGGL(k_cells2<R>, gc, b, 0, s, m, ctl, sc, sn, w.geo, w.r2);
  hipLaunchKernelGGL(k_nodes2<R>, gn, b, 0, s, m, ctl, sc, sn, w.geo, w.up, w.vp, w.wp, w.r2);
  hipLaunchKernelGGL(k_fix2<R>, dim3((unsigned)gf.blocks()), dim3(FW * FH), 0, s, m, ctl, sc, sn, w.r2, gf);
  return hipGetLastError();
}

template hipError_t launch_remap2<double>(const Mesh &, Ctl *, const Work<double> &, int, hipStream_t);
template hipError_t launch_remap2<float>(const Mesh &, Ctl *, const Work<float> &, int, hipStream_t);

}  // namespace sale
