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
// The step's Lagrange kernel hands over rho^L as well (its tile's fifth
// phase); then three passes, each a tile of columns marched along z (every
// input value read from memory once per tile, neighbours through LDS):
//   k_cells2  fluxes through each cell's six faces, M, rho^{n+1}, e^pre
//   k_nodes2  dual fluxes, reconstructed donor velocities, u^{n+1}, KE defect
//   k_fix2    KE fix, e^{n+1}, the next signal speed (block max -> ctl)
// A step after t_end or after an error flag copies the state instead.
#include "sale_tiles.h"

namespace sale {
namespace {

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


// ---- pass 1: face fluxes, cell masses, densities, pre-fix energies --------------------
// A 36 x 14 tile of cell columns owning 32 x 10 (halo 2 on each side: a
// face's donor profile reaches one cell beyond the donor; the owned columns
// start on a multiple of 32, so every stored row is whole 128-byte lines)
// marched along z over one segment; 512 threads, the 8 spare ones own
// nothing. Each cell forms the fluxes of its lower and upper faces on all
// three axes; a face shared by two cells is formed by both from the same
// operands, so both get the same bits. The LDS holds rho^L, e^L and the x/y
// swept volumes of the cell plane; rho^L and e^L of cell planes k-2..k+2 (the
// z profiles) are carried in registers. Stores the lower faces' mass fluxes
// (for the node pass), M, rho^{n+1} and e^pre.
constexpr int CW2 = 36, CH2 = 14, CTX = CW2 - 4, CTY = CH2 - 4;
constexpr int NT2 = (CW2 * CH2 + 63) / 64 * 64, CH2L = (NT2 + CW2 - 1) / CW2;  // threads; LDS rows

template <typename R>
__global__ __launch_bounds__(NT2) void k_cells2(Mesh m, Ctl *ctl, State<R> cur, State<R> nxt, Geo<R> geo,
                                              Rem2<R> t, Grid2 g) {
  enum { RL, EL, DX, DY, NPL };
  __shared__ R L[NPL][CH2L][CW2];  // (row CH2: the spare threads' own, never read)
  int tx, ty, seg;
  tile_of(g, blockIdx.x, tx, ty, seg);
  const int ci = threadIdx.x % CW2, cj = threadIdx.x / CW2;  // cj == CH2: a spare thread
  const int gi = tx * CTX + ci - 2, gj = ty * CTY + cj - 2;  // cell column
  const int Z0 = seg * g.seglen;
  const int Z1 = seg == g.nseg - 1 ? m.nz : Z0 + g.seglen;  // cell planes [Z0, Z1)
  const bool ccol = cj < CH2 && gi >= 0 && gi < m.nx && gj >= 0 && gj < m.ny;
  const bool own = ci >= 2 && cj >= 2 && ci < 2 + CTX && cj < 2 + CTY && ccol;
  const int64_t cpl = (int64_t)m.nx * m.ny;
  const int64_t cix = ccol ? gi + (int64_t)m.nx * gj : 0;
  if (ctl->done) {  // uniform: the state is carried over
    if (own)
      for (int k = Z0; k < Z1; k++) nxt.rho[cix + k * cpl] = cur.rho[cix + k * cpl];
    return;
  }
  // 1 / (h A): the slab's thickness over the spacing is |dv| / (h A)
  const R ihA[3] = {R(1) / (R(m.dx) * R(m.hyz)), R(1) / (R(m.dy) * R(m.hzx)), R(1) / (R(m.dz) * R(m.hxy))};

  // rho^L, e^L of the column at cell planes k-2..k+2, z swept volumes of
  // planes k, k+1 (the cell's lower and upper z faces); zero outside the mesh
  R zr[5], ze[5], zv0, zv1;
  auto lag_load = [&](int p, R &r, R &e) {
    r = e = R(0);
    if (ccol && p >= 0 && p < m.nz) {
      r = geo.rl[cix + p * cpl];
      e = geo.el[cix + p * cpl];
    }
  };
  auto dvz_load = [&](int p) { return ccol && p >= 0 && p < m.nz ? geo.dvz[cix + p * cpl] : R(0); };
  R f_dx = 0, f_dy = 0, f_rho = 0;  // x/y swept volumes and old density of the plane
  auto plane_load = [&](int p) {
    f_dx = f_dy = f_rho = R(0);
    if (ccol && p >= 0 && p < m.nz) {
      const int64_t c = cix + p * cpl;
      f_dx = geo.dvx[c];
      f_dy = geo.dvy[c];
      f_rho = cur.rho[c];
    }
  };
  for (int q = 0; q < 5; q++) lag_load(Z0 - 2 + q, zr[q], ze[q]);
  zv0 = dvz_load(Z0);
  zv1 = dvz_load(Z0 + 1);
  plane_load(Z0);

  // flux of mass and internal energy through a face: donor lower (dv > 0) or
  // upper cell, its values (mean rm/r0/rp of the donor and its neighbours
  // along the axis) taken from the limited linear profile when both
  // neighbours exist (donor index di in [1, n-2])
  auto flux = [&](R dv, int di, int n, R ih, R rm, R r0, R rp, R em, R e0, R ep, R &mu, R &eps) {
    const bool lower = dv > R(0);
    R rf = r0, ef = e0;
    if (di >= 1 && di + 1 < n) {
      const R wgt = donor_weight(dv, ih);
      rf = donor_value(r0, vanleer(r0 - rm, rp - r0), wgt, lower);
      ef = donor_value(e0, vanleer(e0 - em, ep - e0), wgt, lower);
    }
    mu = rf * dv;
    eps = mu * ef;
  };
  // x or y face between LDS cells (x - dx, y - dy) and (x, y); gf is the
  // global index of the upper cell along the axis (walls at 0 and n)
  auto face_xy = [&](int ax, int x, int y, int gf, R &mu, R &eps) {
    const int n = ax == 0 ? m.nx : m.ny;
    mu = eps = R(0);
    if (gf <= 0 || gf >= n) return;
    const int dx = ax == 0, dy = ax == 1;
    const R dv = L[ax == 0 ? DX : DY][y][x];
    const bool lower = dv > R(0);
    const int xd = lower ? x - dx : x, yd = lower ? y - dy : y;
    flux(dv, lower ? gf - 1 : gf, n, ihA[ax], L[RL][yd - dy][xd - dx], L[RL][yd][xd], L[RL][yd + dy][xd + dx],
         L[EL][yd - dy][xd - dx], L[EL][yd][xd], L[EL][yd + dy][xd + dx], mu, eps);
  };

  for (int k = Z0; k < Z1; k++) {
    L[RL][cj][ci] = zr[2];
    L[EL][cj][ci] = ze[2];
    L[DX][cj][ci] = f_dx;
    L[DY][cj][ci] = f_dy;
    const R rho = f_rho;
    // next pass: plane k+1, z swept volume of k+2, rho^L / e^L of k+3
    R nr, ne;
    plane_load(k + 1);
    const R zv2 = dvz_load(k + 2);
    lag_load(k + 3, nr, ne);
    __syncthreads();
    if (own) {
      R mxl, exl, mxu, exu, myl, eyl, myu, eyu;
      face_xy(0, ci, cj, gi, mxl, exl);
      face_xy(0, ci + 1, cj, gi + 1, mxu, exu);
      face_xy(1, ci, cj, gj, myl, eyl);
      face_xy(1, ci, cj + 1, gj + 1, myu, eyu);
      R mzl = R(0), ezl = R(0), mzu = R(0), ezu = R(0);
      if (k > 0) {  // lower z face: donor k-1 (window slot 1) or k (slot 2)
        if (zv0 > R(0))
          flux(zv0, k - 1, m.nz, ihA[2], zr[0], zr[1], zr[2], ze[0], ze[1], ze[2], mzl, ezl);
        else
          flux(zv0, k, m.nz, ihA[2], zr[1], zr[2], zr[3], ze[1], ze[2], ze[3], mzl, ezl);
      }
      if (k + 1 < m.nz) {  // upper z face: donor k (slot 2) or k+1 (slot 3)
        if (zv1 > R(0))
          flux(zv1, k, m.nz, ihA[2], zr[1], zr[2], zr[3], ze[1], ze[2], ze[3], mzu, ezu);
        else
          flux(zv1, k + 1, m.nz, ihA[2], zr[2], zr[3], zr[4], ze[2], ze[3], ze[4], mzu, ezu);
      }
      const R netm = ((mxu - mxl) + (myu - myl)) + (mzu - mzl);
      const R nete = ((exu - exl) + (eyu - eyl)) + (ezu - ezl);
      const R M = rho * R(m.V0) - netm;
      const R rn = rho - netm * R(m.iV0);
      R epre = R(0);
      if (!(M > R(0)) || !(rn > R(0)) || !isfinite(rn)) {
        atomicOr(&ctl->status, SALE_FLAG_NUMERIC);
      } else {
        const R el = ze[2];
        epre = el + (el * netm - nete) / M;
      }
      const int64_t c = cix + k * cpl;
      t.mu[0][c] = mxl;
      t.mu[1][c] = myl;
      t.mu[2][c] = mzl;
      nxt.rho[c] = rn;
      t.M[c] = M;
      t.epre[c] = epre;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; q++) {
      zr[q] = zr[q + 1];
      ze[q] = ze[q + 1];
    }
    zr[4] = nr;
    ze[4] = ne;
    zv0 = zv1;
    zv1 = zv2;
  }
}

// ---- pass 2: node momentum and kinetic-energy remap ------------------------------------
// A 32 x 16 tile of node columns (halo 2 on each side: the limited profiles
// along x and y reach two nodes out) marched along z over one segment. For
// node plane k the LDS holds u' of the plane and the face data of cell
// planes k-1 and k: x/y mass fluxes and swept volumes and the old and new
// cell masses as per-column sums of the two planes (every stencil adds both
// planes), the z faces' lower + upper sums of plane k (those of plane k-1
// are carried in registers, formed in the previous pass). u' of node planes
// k-2..k+2 (the z profiles) is carried in registers. Each input value is
// read from memory once per tile, and each dual edge's flux is evaluated once
// (by its lower node; the in-plane ones are handed to the upper node through
// LDS, the z one to the next plane in registers).
// (36 x 14 tiles owning 32 x 10 nodes ran slower here: 1.32 -> 1.44 ms at
// 320^3; the node arrays' rows do not start on 128-byte lines anyway)
constexpr int NW = 32, NH = 16;
constexpr int NTX = NW - 4, NTY = NH - 4;
constexpr int NT3 = (NW * NH + 63) / 64 * 64, NHL = (NT3 + NW - 1) / NW;  // threads; LDS rows

template <typename R>
__global__ __launch_bounds__(NT3, 4) void k_nodes2(Mesh m, Ctl *ctl, State<R> cur, State<R> nxt, Geo<R> geo,
                                               const R *up, const R *vp, const R *wp, Rem2<R> t, Grid2 g) {
  enum { MX, MY, VX, VY, SZ, VZ, MO, MN, NCP };
  __shared__ R LU[3][NHL][NW];    // u', v', w' of node plane k
  __shared__ R LC[NCP][NHL][NW];  // MX..VY, MO, MN: cell planes k-1 + k; SZ, VZ: plane k
  __shared__ R LP[6][NHL][NW];    // the thread's own column at cell plane k-1 (private)
  // (row NH of each: the spare threads' own, never read by a stencil)
  int tx, ty, seg;
  tile_of(g, blockIdx.x, tx, ty, seg);
  const int ci = threadIdx.x % NW, cj = threadIdx.x / NW;  // cj == NH: a spare thread
  const int gi = tx * NTX + ci - 2, gj = ty * NTY + cj - 2;  // node column, and cell column (gi, gj)
  const int Z0 = seg * g.seglen;
  const int NZ1 = seg == g.nseg - 1 ? m.nz + 1 : Z0 + g.seglen;  // node planes [Z0, NZ1)
  const bool ncol = cj < NH && gi >= 0 && gi <= m.nx && gj >= 0 && gj <= m.ny;
  const bool ccol = cj < NH && gi >= 0 && gi < m.nx && gj >= 0 && gj < m.ny;
  const bool own = ci >= 2 && cj >= 2 && ci < 2 + NTX && cj < 2 + NTY && gi <= m.nx && gj <= m.ny;
  const int64_t cpl = (int64_t)m.nx * m.ny, npl = (int64_t)(m.nx + 1) * (m.ny + 1);
  const int64_t cix = ccol ? gi + (int64_t)m.nx * gj : 0, nix = ncol ? gi + (int64_t)(m.nx + 1) * gj : 0;
  if (ctl->done) {  // uniform: the state is carried over
    if (own)
      for (int k = Z0; k < NZ1; k++) {
        const int64_t q = nix + k * npl;
        nxt.u[q] = cur.u[q];
        nxt.v[q] = cur.v[q];
        nxt.w[q] = cur.w[q];
      }
    return;
  }
  const R ihA[3] = {R(1) / (R(m.dx) * R(m.hyz)), R(1) / (R(m.dy) * R(m.hzx)), R(1) / (R(m.dz) * R(m.hxy))};
  const R V0 = R(m.V0);

  // u' of the column at node planes k-2..k+2 (zero outside the mesh)
  R zu[5], zv[5], zw[5];
  auto node_load = [&](int p, R &u, R &v, R &w) {
    u = v = w = R(0);
    if (ncol && p >= 0 && p <= m.nz) {
      const int64_t q = nix + p * npl;
      u = up[q];
      v = vp[q];
      w = wp[q];
    }
  };
  // face data of the column's cell at plane p (zero outside the mesh)
  R f_mx, f_my, f_vx, f_vy, f_mo, f_mn;  // cell plane k+1
  R z_m1, z_v1, z_m2, z_v2;              // z-face flux, swept volume of cell planes k+1, k+2
  auto cell_load = [&](int p) {
    f_mx = f_my = f_vx = f_vy = f_mo = f_mn = R(0);
    if (ccol && p >= 0 && p < m.nz) {
      const int64_t c = cix + p * cpl;
      f_mx = t.mu[0][c];
      f_my = t.mu[1][c];
      f_vx = geo.dvx[c];
      f_vy = geo.dvy[c];
      f_mo = cur.rho[c] * V0;
      f_mn = t.M[c];
    }
  };
  auto zface_load = [&](int p, R &mz, R &vz) {
    mz = vz = R(0);
    if (ccol && p >= 0 && p < m.nz) {
      const int64_t c = cix + p * cpl;
      mz = t.mu[2][c];
      vz = geo.dvz[c];
    }
  };
  const int K0 = Z0 - 1;  // first pass: sums of cell plane Z0-1 for node plane Z0
  for (int q = 0; q < 5; q++) node_load(K0 - 2 + q, zu[q], zv[q], zw[q]);
  cell_load(K0 - 1);
  LP[0][cj][ci] = f_mx;
  LP[1][cj][ci] = f_my;
  LP[2][cj][ci] = f_vx;
  LP[3][cj][ci] = f_vy;
  LP[4][cj][ci] = f_mo;
  LP[5][cj][ci] = f_mn;
  cell_load(K0);
  R z_m0, z_v0;
  zface_load(K0, z_m0, z_v0);
  zface_load(K0 + 1, z_m1, z_v1);

  // the z dual faces below node plane k (those of cell plane k-1), carried
  // from the previous pass
  R zl[4] = {R(0), R(0), R(0), R(0)};
  for (int k = K0; k < NZ1; k++) {
    R(*const C)[NHL][NW] = LC;
    LU[0][cj][ci] = zu[2];
    LU[1][cj][ci] = zv[2];
    LU[2][cj][ci] = zw[2];
    // every stencil below sums a field over the cells of planes k-1 and k
    // around the node: the two planes are added per cell column here
    C[MX][cj][ci] = LP[0][cj][ci] + f_mx;
    C[MY][cj][ci] = LP[1][cj][ci] + f_my;
    C[VX][cj][ci] = LP[2][cj][ci] + f_vx;
    C[VY][cj][ci] = LP[3][cj][ci] + f_vy;
    C[SZ][cj][ci] = z_m0 + z_m1;  // lower + upper z face of the cell
    C[VZ][cj][ci] = z_v0 + z_v1;
    C[MO][cj][ci] = LP[4][cj][ci] + f_mo;
    C[MN][cj][ci] = LP[5][cj][ci] + f_mn;
    LP[0][cj][ci] = f_mx;
    LP[1][cj][ci] = f_my;
    LP[2][cj][ci] = f_vx;
    LP[3][cj][ci] = f_vy;
    LP[4][cj][ci] = f_mo;
    LP[5][cj][ci] = f_mn;
    // next pass: cell plane k+1, z faces of k+2, node plane k+3
    R nu, nv, nw;
    cell_load(k + 1);
    zface_load(k + 2, z_m2, z_v2);
    node_load(k + 3, nu, nv, nw);
    __syncthreads();
    // sums over the 4 cell columns around the node (zero where absent)
    auto c4 = [&](R(*P)[NHL][NW], int s) {
      return ((P[s][cj - 1][ci - 1] + P[s][cj - 1][ci]) + P[s][cj][ci - 1]) + P[s][cj][ci];
    };
    // the z dual faces above node plane k: those of the 4 cells of plane k
    const R za_m = own ? R(0.125) * c4(C, SZ) : R(0), za_v = own ? R(0.125) * c4(C, VZ) : R(0);
    // Every dual edge is evaluated once: an in-plane edge by its lower node
    // (the out-edge; the upper node takes it as its in-edge from LDS), a z edge
    // at its lower node plane (carried to the next plane as that plane's lower
    // edge). An edge's contribution is (phi u_d, phi v_d, phi w_d,
    // phi |u_d|^2 / 2) with the donor's limited linear values u_d; the out-node
    // subtracts it, the in-node adds it.
    // donor value of one component: limited linear profile of the donor
    // (values qm, q0, qp at the donor and its two neighbours along the edge)
    auto recon = [&](R qm, R q0, R qp, bool both, R wgt, bool plus) {
      return both ? donor_value(q0, vanleer(q0 - qm, qp - q0), wgt, plus) : q0;
    };
    auto contrib = [&](R phi, R ud, R vd, R wd, R *e) {
      e[0] = phi * ud;
      e[1] = phi * vd;
      e[2] = phi * wd;
      e[3] = phi * R(0.5) * (ud * ud + vd * vd + wd * wd);
    };
    // in-plane edge along x (ax 0) or y (ax 1) from the node at global index
    // glo (this column) to glo + 1
    auto inplane = [&](int ax, int nlim, int glo, R phi, R dv, R *e) {
      const bool lower = phi > R(0);
      const int dg = lower ? glo : glo + 1;
      const bool both = dg >= 1 && dg + 1 <= nlim;
      const R wgt = donor_weight(dv, ihA[ax]);
      const bool plus = lower && dv != R(0);
      const int dx = ax == 0, dy = ax == 1;
      const int x0 = ci + (ax == 0 ? dg - gi : 0), y0 = cj + (ax == 1 ? dg - gj : 0);
      const R ud = recon(LU[0][y0 - dy][x0 - dx], LU[0][y0][x0], LU[0][y0 + dy][x0 + dx], both, wgt, plus);
      const R vd = recon(LU[1][y0 - dy][x0 - dx], LU[1][y0][x0], LU[1][y0 + dy][x0 + dx], both, wgt, plus);
      const R wd = recon(LU[2][y0 - dy][x0 - dx], LU[2][y0][x0], LU[2][y0 + dy][x0 + dx], both, wgt, plus);
      contrib(phi, ud, vd, wd, e);
    };
    // the out-edges along x of columns 1 .. NTX+1 and along y of rows 1 ..
    // NTY+1 of the owned range (the first halo column / row gives the owned
    // nodes' in-edges)
    const bool inx = ci >= 2 && ci < 2 + NTX, iny = cj >= 2 && cj < 2 + NTY;
    const bool xcomp = ncol && ci >= 1 && ci < 2 + NTX && iny && gi + 1 <= m.nx && k >= Z0;
    const bool ycomp = ncol && cj >= 1 && cj < 2 + NTY && inx && gj + 1 <= m.ny && k >= Z0;
    R ex[4] = {R(0), R(0), R(0), R(0)}, ey[4] = {R(0), R(0), R(0), R(0)}, ez[4] = {R(0), R(0), R(0), R(0)};
    if (xcomp) {
      // cells (i, j-1..j) of planes k-1 and k
      const R phi = R(0.125) * ((C[MX][cj - 1][ci] + C[MX][cj - 1][ci + 1]) + (C[MX][cj][ci] + C[MX][cj][ci + 1]));
      const R dv = R(0.125) * ((C[VX][cj - 1][ci] + C[VX][cj - 1][ci + 1]) + (C[VX][cj][ci] + C[VX][cj][ci + 1]));
      inplane(0, m.nx, gi, phi, dv, ex);
    }
    if (ycomp) {
      // cells (i-1..i, j)
      const R phi = R(0.125) * ((C[MY][cj][ci - 1] + C[MY][cj + 1][ci - 1]) + (C[MY][cj][ci] + C[MY][cj + 1][ci]));
      const R dv = R(0.125) * ((C[VY][cj][ci - 1] + C[VY][cj + 1][ci - 1]) + (C[VY][cj][ci] + C[VY][cj + 1][ci]));
      inplane(1, m.ny, gj, phi, dv, ey);
    }
    // the z edge from node plane k to k+1 (its dual face is that of the 4
    // cells of plane k); the column's u' at node planes k-2..k+2 is window
    // slots 0..4
    if (own && k + 1 <= m.nz) {
      const bool lower = za_m > R(0);
      const int dg = lower ? k : k + 1;  // donor's node plane
      const bool both = dg >= 1 && dg + 1 <= m.nz;
      const R wgt = donor_weight(za_v, ihA[2]);
      const bool plus = lower && za_v != R(0);
      R ud, vd, wd;
      if (lower) {  // donor plane k: slots 1..3
        ud = recon(zu[1], zu[2], zu[3], both, wgt, plus);
        vd = recon(zv[1], zv[2], zv[3], both, wgt, plus);
        wd = recon(zw[1], zw[2], zw[3], both, wgt, plus);
      } else {  // donor plane k+1: slots 2..4
        ud = recon(zu[2], zu[3], zu[4], both, wgt, plus);
        vd = recon(zv[2], zv[3], zv[4], both, wgt, plus);
        wd = recon(zw[2], zw[3], zw[4], both, wgt, plus);
      }
      contrib(za_m, ud, vd, wd, ez);
    }
    const bool fin = own && k >= Z0;
    const R mp = fin ? R(0.125) * (c4(C, MO)) : R(0), mn = fin ? R(0.125) * (c4(C, MN)) : R(0);
    __syncthreads();  // the cell sums are read: their planes take the out-edges
    C[0][cj][ci] = ex[0];
    C[1][cj][ci] = ex[1];
    C[2][cj][ci] = ex[2];
    C[3][cj][ci] = ex[3];
    C[4][cj][ci] = ey[0];
    C[5][cj][ci] = ey[1];
    C[6][cj][ci] = ey[2];
    C[7][cj][ci] = ey[3];
    __syncthreads();
    if (fin) {
      const R u1 = zu[2], v1 = zv[2], w1 = zw[2];
      R P0 = mp * u1, P1 = mp * v1, P2 = mp * w1;
      R K = R(0.5) * mp * (u1 * u1 + v1 * v1 + w1 * w1);
      auto add = [&](R a0, R a1, R a2, R a3, R sgn) {
        P0 += sgn * a0;
        P1 += sgn * a1;
        P2 += sgn * a2;
        K += sgn * a3;
      };
      if (gi + 1 <= m.nx) add(ex[0], ex[1], ex[2], ex[3], R(-1));  // x out
      if (gi >= 1) add(C[0][cj][ci - 1], C[1][cj][ci - 1], C[2][cj][ci - 1], C[3][cj][ci - 1], R(1));  // x in
      if (gj + 1 <= m.ny) add(ey[0], ey[1], ey[2], ey[3], R(-1));  // y out
      if (gj >= 1) add(C[4][cj - 1][ci], C[5][cj - 1][ci], C[6][cj - 1][ci], C[7][cj - 1][ci], R(1));  // y in
      if (k + 1 <= m.nz) add(ez[0], ez[1], ez[2], ez[3], R(-1));  // z out
      if (k >= 1) add(zl[0], zl[1], zl[2], zl[3], R(1));          // z in (carried)
      R un = R(0), vn = R(0), wn = R(0), dk = R(0);
      if (!(mn > R(0))) {
        atomicOr(&ctl->status, SALE_FLAG_NUMERIC);
      } else {
        const R imn = R(1) / mn;
        un = P0 * imn;
        vn = P1 * imn;
        wn = P2 * imn;
        if (gi == 0 || gi == m.nx) un = R(0);
        if (gj == 0 || gj == m.ny) vn = R(0);
        if (k == 0 || k == m.nz) wn = R(0);
        dk = (K - R(0.5) * mn * (un * un + vn * vn + wn * wn)) * imn;
      }
      const int64_t q = nix + k * npl;
      nxt.u[q] = un;
      nxt.v[q] = vn;
      nxt.w[q] = wn;
      t.dk[q] = dk;
    }
#pragma unroll
    for (int q = 0; q < 4; q++) zl[q] = ez[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; q++) {
      zu[q] = zu[q + 1];
      zv[q] = zv[q + 1];
      zw[q] = zw[q + 1];
    }
    zu[4] = nu;
    zv[4] = nv;
    zw[4] = nw;
    z_m0 = z_m1;
    z_v0 = z_v1;
    z_m1 = z_m2;
    z_v1 = z_v2;
  }
}

// ---- pass 3: kinetic-energy fix, new energy, next signal speed ------------------------
// A 33 x 15 tile of node columns (512 threads, 17 spare) owning 32 x 14
// cells, marched along z over one segment: each node plane's u^{n+1}, v, w
// and KE defect are read once into LDS, a cell column forms its lower-plane
// half (partial defect sum, largest |u|^2, divergence halves) and finishes
// the cell when the upper plane arrives. Sums run in the order of the
// cell's 8 nodes (x fastest, then y, then z), as in the gather form of the
// same pass. The owned cells of a row start on a multiple of 32, so the
// stored energies fill whole 128-byte lines.
constexpr int FW = 33, FH = 15;
constexpr int FTX = FW - 1, FTY = FH - 1;
constexpr int NT4 = (FW * FH + 63) / 64 * 64, FHL = (NT4 + FW - 1) / FW;  // threads; LDS rows

template <typename R>
__global__ __launch_bounds__(NT4) void k_fix2(Mesh m, Ctl *ctl, State<R> cur, State<R> nxt, Rem2<R> t, Grid2 g) {
  __shared__ R sU[FHL][FW], sV[FHL][FW], sW[FHL][FW], sQ[FHL][FW];  // (row FH: the spare threads')
  int tx, ty, seg;
  tile_of(g, blockIdx.x, tx, ty, seg);
  const int ci = threadIdx.x % FW, cj = threadIdx.x / FW;  // cj == FH: a spare thread
  const int gi = tx * FTX + ci, gj = ty * FTY + cj;  // node column; cell column when owned
  const int Z0 = seg * g.seglen;
  const int Z1 = seg == g.nseg - 1 ? m.nz : Z0 + g.seglen;  // cell planes [Z0, Z1)
  const bool ncol = cj < FH && gi <= m.nx && gj <= m.ny;
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
  block_max_to_ctl<NT4>(ctl, a, bad);
}

}  // namespace

template <typename R>
hipError_t launch_remap2(const Mesh &m, Ctl *ctl, const Work<R> &w, int cur, hipStream_t s) {
  if (m.order != 2 || !w.r2.M || !w.geo.rl) return hipErrorInvalidValue;
  const State<R> sc = w.s[cur], sn = w.s[1 - cur];
  // tiles of the three passes: about 6144 blocks, at least 8
  // planes per z segment
  auto tiles = [](int cols, int rows, int planes, int tw, int th) {
    Grid2 g;
    g.tx = (cols + tw - 1) / tw;
    g.ty = (rows + th - 1) / th;
    const int maxseg = planes / 8 > 1 ? planes / 8 : 1;
    int nseg = (6144 + g.tx * g.ty / 2) / (g.tx * g.ty);
    nseg = nseg < 1 ? 1 : nseg > maxseg ? maxseg : nseg;
    g.seglen = (planes + nseg - 1) / nseg;
    g.nseg = (planes + g.seglen - 1) / g.seglen;
    return g;
  };
  const Grid2 gnode = tiles(m.nx + 1, m.ny + 1, m.nz + 1, NTX, NTY);
  const Grid2 gf = tiles(m.nx, m.ny, m.nz, FTX, FTY);
  const Grid2 gcell = tiles(m.nx, m.ny, m.nz, CTX, CTY);
  hipLaunchKernelGGL(k_cells2<R>, dim3((unsigned)gcell.blocks()), dim3(NT2), 0, s, m, ctl, sc, sn, w.geo, w.r2,
                     gcell);
  hipLaunchKernelGGL(k_nodes2<R>, dim3((unsigned)gnode.blocks()), dim3(NT3), 0, s, m, ctl, sc, sn, w.geo, w.up,
                     w.vp, w.wp, w.r2, gnode);
  hipLaunchKernelGGL(k_fix2<R>, dim3((unsigned)gf.blocks()), dim3(NT4), 0, s, m, ctl, sc, sn, w.r2, gf);
  return hipGetLastError();
}

template hipError_t launch_remap2<double>(const Mesh &, Ctl *, const Work<double> &, int, hipStream_t);
template hipError_t launch_remap2<float>(const Mesh &, Ctl *, const Work<float> &, int, hipStream_t);

}  // namespace sale
