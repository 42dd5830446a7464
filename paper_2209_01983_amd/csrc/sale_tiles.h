// sale_tiles.h -- the two z-marching tile functions of the SALE step, shared
// by the single-run kernels and the persistent multi-run kernel.
//
// One step is the Lagrangian phase on the structured hex mesh followed by the
// Eulerian rezone and donor-cell advection back to the fixed mesh (ScalSALE
// Sec. I-D and Table I: "Lagrangian rezoning", "Eulerian rezoning",
// "Advection"), with the ideal-gas EoS (Sec. I-C/I-D), cell-centred rho/e/p/q
// and vertex velocities (Sec. III-C/III-D) and density as mass over volume
// (Sec. III-A). The paper prints no scheme equations; the tiles compute the
// scheme of the project's FP64 oracle (its steps O1..O12):
//
//   lagrange_tile  O1, O2, O4..O8  EOS, divergence, viscosity, acoustic
//                  predictor P*, atomic-free gather of corner forces, u',
//                  walls, compatible energy e^L, exact swept volumes, V^L, rho^L
//   remap_tile     O9..O11 and the next O3 reduction: donor-cell face fluxes,
//                  M, rho^{n+1}, e^pre, dual-mesh momentum / KE remap,
//                  u^{n+1}, KE fix, e^{n+1}, next signal speed
//
// A tile is a kTileW x CH grid of (x, y) columns (36 x 14 by default), one
// thread per column, marched along z over one z segment one plane at a time. A plane's values live in
// LDS while its x/y neighbours need them; values a column needs again one or
// two planes later stay in that column's registers; global loads run one
// plane ahead. The hand-off between the two tiles is u' (per node) and the
// Lagrangian cell results rho^L, e^L and three lower-face swept volumes,
// whose faces need only the cell's own nodes, so no geometry is computed
// twice. Nothing scatters, so results do not depend on scheduling.
//
// Precision: R is the bulk type (double, or float for SALE_MIXED32). Node
// displacements, swept volumes, volume differences and V^L are always
// computed in double, as are dt and the signal-speed reduction.
#pragma once

#include <type_traits>

#include "sale_device.h"

namespace sale {

// Element of plane k of a plane-major array (`plane` elements per z plane) at
// the in-plane byte offset `off`: the plane base is uniform (scalar
// registers), the offset a 32-bit per-thread value, so a load or store needs
// no per-thread 64-bit address arithmetic.
template <typename T>
__device__ __forceinline__ T &plane_at(T *base, int64_t plane, int k, uint32_t off) {
  const uint32_t b = (uint32_t)(plane * (int64_t)k * (int64_t)sizeof(T)) + off;
  return *reinterpret_cast<T *>(reinterpret_cast<
      typename std::conditional<std::is_const<T>::value, const char, char>::type *>(base) + (uint64_t)b);
}

// A prefetched value is settled here: the wait for its load is taken at this
// point, and later uses see a value produced by the (empty) statement, so
// they wait for nothing. The hardware counts loads and stores in one counter
// and the compiler, across branches, can only wait for all of them at once:
// a value used first at the top of the next plane would drain that plane's
// stores as well, and one loaded before the loop would drain the loads just
// issued. Settling a plane's prefetch after its longest phase and before its
// stores keeps both off the critical path.
template <typename T>
__device__ __forceinline__ void settle(T &x) {
  asm volatile("" : "+v"(x));
}

// ---- O5: acoustic predictor P* of one cell (O2, O4 folded in) ----------------
// Divisions by a quantity used more than once go through one reciprocal
// (rounding-level differences from the oracle's divisions).
template <typename R>
__device__ __forceinline__ R predict_ps(const Mesh &m, R rho, R e, R D, R dt, bool &tangle, R &inv_mc) {
  const R V0 = R(m.V0), h = R(m.h), gm1 = R(m.gm1);
  const R mc = rho * V0;
  const R p = gm1 * rho * e;
  const R cs = sqrt(R(m.ggm1) * fmax(e, R(0)));
  R q = R(0);
  if (D < R(0)) {
    const R hd = h * D;
    q = rho * (R(m.cq) * hd * hd + R(m.cl) * cs * h * fabs(D));
  }
  const R dVs = R(0.5) * dt * V0 * D;
  const R Vs = V0 + dVs;
  if (!(Vs > R(0))) {
    tangle = true;
    return R(0);
  }
  inv_mc = R(1) / mc;
  const R rs = mc / Vs;
  const R es = e - (p + q) * dVs * inv_mc;
  return gm1 * rs * es + q;
}

// ---- O3: signal speed from a cell's divergence, energy and node speeds --------
template <typename R>
__device__ __forceinline__ R signal_from(const Mesh &m, R D, R e, R smax) {
  const R cs = sqrt(R(m.ggm1) * fmax(e, R(0)));
  return fma(R(m.cq4h), fmax(-D, R(0)), cs + smax);
}

// O3 at the start of a step: dt from the largest signal speed of the current
// state (CFL h / a_max, clipped to land on t_end) and the done decision (error
// flag raised, t_end reached, or the run's step target reached). Run by one
// thread; every kernel of the step then reads ctl->dt and ctl->done.
__device__ __forceinline__ void begin_step(const Mesh &m, Ctl *ctl, long long step_target) {
  if (ctl->status != 0u || ctl->t >= ctl->t_end || ctl->step >= step_target) {
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

__device__ __forceinline__ void tile_of(const Grid2 &g, int b, int &tx, int &ty, int &seg) {
  tx = b % g.tx;
  const int r = b / g.tx;
  ty = r % g.ty;
  seg = r / g.ty;
}

// Tile geometry. A tile is CW columns in x by CH rows in y, of which
// kTileX = 32 in x are owned: a row of a tile's owned cells is a whole number
// of 128-byte lines (32 doubles or floats, on meshes whose x extent is a
// multiple of 16 cells), so neighbouring tiles never write parts of the same
// line (a line written in parts by two blocks costs the memory system far
// more than whole lines) and 320 cells split into 10 tiles. The halo makes
// the Lagrange tile kTileWL = 35 columns wide (one below, two above) and the
// remap tile kTileW = 36 (two on each side). A block rounds 36 x CH threads
// up to a multiple of 64 (tile_threads); the spare threads map to LDS rows CH
// and beyond of their own and own nothing, so every wave is whole and every
// thread meets every barrier. The tile width is a template parameter: the
// multi-run kernels, whose meshes are 16-64 cells across, keep tiles 32
// columns wide (29 and 28 owned), which waste less of a small mesh.
constexpr int kTileW = 36, kTileWL = 35, kTileX = 32;
template <int CH, int CW = kTileW>
constexpr int tile_threads() {
  return (CW * CH + 63) / 64 * 64;
}
// rows of an LDS plane of a CW-wide tile in a block of NT threads: CH and the
// spare threads' rows
template <int CW, int CH, int NT>
constexpr int lds_rows() {
  return (NT + CW - 1) / CW;
}

// LDS doubles needed by each tile function (planes of CW x lds_rows) in a
// block of NT threads (RL: the Lagrange tile that also forms rho^L)
template <int CH, int CW = kTileWL, int NT = tile_threads<CH>(), bool RL = false>
constexpr int lagrange_lds_doubles() {
  return (RL ? 13 : 11) * CW * lds_rows<CW, CH, NT>();
}
// (remap: two double planes, then 16 planes of the bulk type R)
template <typename R, int CH, int CW = kTileW, int NT = tile_threads<CH>()>
constexpr int remap_lds_doubles() {
  return (2 * 8 + 16 * (int)sizeof(R)) * CW * lds_rows<CW, CH, NT>() / 8;
}

// ---------------------------------------------------------------------------------
// lagrange_tile: the Lagrangian phase of one tile
// ---------------------------------------------------------------------------------
// Column (ci, cj) is node column / cell column (X0 + ci - 1, Y0 + cj - 1). The
// tile owns cells [X0, X0+TX) x [Y0, Y0+TY) of its z segment and the matching
// nodes (TX = 32, TY = CH - 3; halo one column below and two above).
// Iteration k:
//   P1  u of node plane k+1 into LDS (loaded one iteration earlier)
//   P2  D and P* of cell plane k (halo 1): the divergence sums edge
//       differences of u over the cell's two node planes; each node plane's
//       half is formed once and carried one plane
//   P3  u' and delta = dt (u + u')/2 of node plane k: gather of P* over the
//       node's 8 cells as a per-plane sum carried one plane            (LDS)
//   P4  swept volumes of the three lower faces of cell plane k-1 (they need
//       delta on node planes k-1 and k only), its compatible-energy work and
//       e^L; hand-off to remap_tile, which forms V^L and rho^L from the six
//       faces' swept volumes
//   P5  (RL only) V^L = V0 + the six faces' swept volumes (FP64) and rho^L
//       of cell plane k-1, the upper x/y faces being the +x/+y neighbours'
//       lower faces (the first halo column and row above form theirs too),
//       for the second-order remap's passes
// Returns true if a tangled cell was seen (the predictor's volume; with RL
// also V^L). CW: tile width, NTH: block size.
template <typename R, int CH, int CW = kTileWL, int NTH = tile_threads<CH>(), bool RL = false>
__device__ bool lagrange_tile(const RunArgs<R> &a, int b, double dtd, double *lds) {
  constexpr int TX = CW - 3, TY = CH - 3, CHL = lds_rows<CW, CH, NTH>();
  static_assert(CW * CH <= NTH, "one thread per column");
  const Mesh &m = a.m;
  const State<R> &cur = a.cur;
  int tx, ty, seg;
  tile_of(a.ga, b, tx, ty, seg);
  const int ci = threadIdx.x % CW, cj = threadIdx.x / CW;  // cj == CH: a spare thread
  const int gi = tx * TX + ci - 1, gj = ty * TY + cj - 1;
  const int Z0 = seg * a.ga.seglen;
  const bool lastseg = seg == a.ga.nseg - 1;
  const int Z1 = lastseg ? m.nz : Z0 + a.ga.seglen;  // cell planes [Z0, Z1)
  const int NZ1 = lastseg ? m.nz + 1 : Z1;           // node planes [Z0, NZ1)
  const bool ncol = cj < CH && gi >= 0 && gi <= m.nx && gj >= 0 && gj <= m.ny;
  const bool inner = ci < CW - 1 && cj < CH - 1;  // has the +x and +y neighbour column
  const bool ccol = inner && gi >= 0 && gi < m.nx && gj >= 0 && gj < m.ny;
  const bool nodecol = ci >= 1 && cj >= 1 && inner;  // u' computed here
  const bool own_node = ncol && ci >= 1 && cj >= 1 && (ci <= TX || gi == m.nx) && (cj <= TY || gj == m.ny);
  const bool own_cell = ci >= 1 && cj >= 1 && ci <= TX && cj <= TY && gi < m.nx && gj < m.ny;
  const int64_t cpl = (int64_t)m.nx * m.ny, npl = (int64_t)(m.nx + 1) * (m.ny + 1);
  const uint32_t cix = ccol ? (uint32_t)(gi + m.nx * gj) : 0u, nix = ncol ? (uint32_t)(gi + (m.nx + 1) * gj) : 0u;

  // LDS: bulk planes as R, delta ring as double
  R(*sU)[CHL][CW] = reinterpret_cast<R(*)[CHL][CW]>(lds);                 // [3]
  R(*sP)[CW] = reinterpret_cast<R(*)[CW]>(lds + 3 * CHL * CW);            // P*
  R(*sM)[CW] = reinterpret_cast<R(*)[CW]>(lds + 4 * CHL * CW);            // m
  double(*sD)[3][CHL][CW] = reinterpret_cast<double(*)[3][CHL][CW]>(lds + 5 * CHL * CW);  // [2][3]
  double(*sVX)[CW] = reinterpret_cast<double(*)[CW]>(lds + 11 * CHL * CW);  // (RL) lower x faces
  double(*sVY)[CW] = reinterpret_cast<double(*)[CW]>(lds + 12 * CHL * CW);  // (RL) lower y faces
  static_assert((RL ? 13 : 11) * CHL * CW <= lagrange_lds_doubles<CH, CW, NTH, RL>(), "lagrange LDS layout");

  for (int q = threadIdx.x; q < 2 * 3 * CHL * CW; q += NTH) (&sD[0][0][0][0])[q] = 0.0;

  const R dt = R(dtd);
  const R ax = R(m.ax), ay = R(m.ay), az = R(m.az), V0 = R(m.V0);
  R pxu = 0, pyu = 0, pzu = 0;       // node-plane halves of D (plane k)
  R fx = 0, fy = 0, fz = 0, mk = 0;  // 4-cell sums of P*, m of cell plane k-1
  R u0 = 0, v0 = 0, w0 = 0;          // own column's u at node plane k
  double pxd = 0.0, pyd = 0.0, pzd = 0.0;  // node-plane halves of the work (plane k-1)
  double dvz_lo = 0.0;                     // z-face swept volume at node plane k-1
  R ps1 = 0, e1 = 0, m1 = 0;               // P*, e, m of cell plane k-1
  bool tangle = false;

  // global loads run one plane ahead
  R fu = 0, fv = 0, fw = 0, frho = 0, fe = 0;
  auto fetch = [&](int k) {
    fu = fv = fw = frho = fe = R(0);
    if (ncol && k + 1 >= 0 && k + 1 <= m.nz) {
      const uint32_t o = nix * (uint32_t)sizeof(R);
      fu = plane_at<const R>(cur.u, npl, k + 1, o);
      fv = plane_at<const R>(cur.v, npl, k + 1, o);
      fw = plane_at<const R>(cur.w, npl, k + 1, o);
    }
    if (ccol && k >= 0 && k < m.nz) {
      const uint32_t o = cix * (uint32_t)sizeof(R);
      frho = plane_at<const R>(cur.rho, cpl, k, o);
      fe = plane_at<const R>(cur.e, cpl, k, o);
    }
  };
  fetch(Z0 - 2);
  settle(fu), settle(fv), settle(fw), settle(frho), settle(fe);

  for (int k = Z0 - 2; k <= Z1; k++) {
    // ---- P1 ----
    const R un = fu, vn = fv, wn = fw, rho_k = frho, e_k = fe;
    fetch(k + 1);
    sU[0][cj][ci] = un;
    sU[1][cj][ci] = vn;
    sU[2][cj][ci] = wn;
    __syncthreads();
    // ---- P2 ----
    R ps = 0, mc = 0, imc = 0;
    {
      R qxu = 0, qyu = 0, qzu = 0;
      if (inner) {
        qxu = (sU[0][cj][ci + 1] - sU[0][cj][ci]) + (sU[0][cj + 1][ci + 1] - sU[0][cj + 1][ci]);
        qyu = (sU[1][cj + 1][ci] - sU[1][cj][ci]) + (sU[1][cj + 1][ci + 1] - sU[1][cj][ci + 1]);
        qzu = ((sU[2][cj][ci] + sU[2][cj][ci + 1]) + sU[2][cj + 1][ci]) + sU[2][cj + 1][ci + 1];
      }
      if (ccol && k >= 0 && k < m.nz) {
        mc = rho_k * V0;
        const R D = divergence(m, pxu, qxu, pyu, qyu, pzu, qzu);
        bool t = false;
        ps = predict_ps(m, rho_k, e_k, D, dt, t, imc);
        if (t && own_cell && k >= Z0 && k < Z1) tangle = true;
      }
      pxu = qxu;
      pyu = qyu;
      pzu = qzu;
    }
    sP[cj][ci] = ps;
    sM[cj][ci] = mc;
    __syncthreads();
    // ---- P3 ----
    {
      double d0 = 0.0, d1 = 0.0, d2 = 0.0;
      if (nodecol) {
        const R gx = (sP[cj][ci - 1] - sP[cj][ci]) + (sP[cj - 1][ci - 1] - sP[cj - 1][ci]);
        const R gy = (sP[cj - 1][ci] - sP[cj][ci]) + (sP[cj - 1][ci - 1] - sP[cj][ci - 1]);
        const R gz = ((sP[cj][ci] + sP[cj][ci - 1]) + sP[cj - 1][ci]) + sP[cj - 1][ci - 1];
        const R gm = ((sM[cj][ci] + sM[cj][ci - 1]) + sM[cj - 1][ci]) + sM[cj - 1][ci - 1];
        if (ncol && k >= 0 && k <= m.nz) {
          // node k is the +z corner of the cells of plane k-1, the -z corner of plane k
          const R Fx = ax * (fx + gx), Fy = ay * (fy + gy), Fz = az * (fz - gz);
          const R mp = R(0.125) * (mk + gm);
          const R dtm = dt / mp;
          R u1 = u0 + dtm * Fx;
          R v1 = v0 + dtm * Fy;
          R w1 = w0 + dtm * Fz;
          if (gi == 0 || gi == m.nx) u1 = R(0);
          if (gj == 0 || gj == m.ny) v1 = R(0);
          if (k == 0 || k == m.nz) w1 = R(0);
          if (own_node && k >= Z0 && k < NZ1) {
            const uint32_t o = nix * (uint32_t)sizeof(R);
            plane_at<R>(a.up, npl, k, o) = u1;
            plane_at<R>(a.vp, npl, k, o) = v1;
            plane_at<R>(a.wp, npl, k, o) = w1;
          }
          d0 = dtd * (0.5 * ((double)u0 + (double)u1));
          d1 = dtd * (0.5 * ((double)v0 + (double)v1));
          d2 = dtd * (0.5 * ((double)w0 + (double)w1));
        }
        fx = gx;
        fy = gy;
        fz = gz;
        mk = gm;
      }
      sD[k & 1][0][cj][ci] = d0;
      sD[k & 1][1][cj][ci] = d1;
      sD[k & 1][2][cj][ci] = d2;
      u0 = un;
      v0 = vn;
      w0 = wn;
    }
    __syncthreads();
    // ---- P4: faces, work and e^L of cell plane k-1 ----
    const int cp = k - 1;
    const bool plane_ok = cp >= 0 && cp < m.nz && k > Z0 - 2;
    {
      const double(*A)[CHL][CW] = sD[cp & 1];  // node plane k-1
      const double(*B)[CHL][CW] = sD[k & 1];   // node plane k
      double qxd = 0.0, qyd = 0.0, qzd = 0.0;
      if (inner) {
        qxd = (B[0][cj][ci + 1] - B[0][cj][ci]) + (B[0][cj + 1][ci + 1] - B[0][cj + 1][ci]);
        qyd = (B[1][cj + 1][ci] - B[1][cj][ci]) + (B[1][cj + 1][ci + 1] - B[1][cj][ci + 1]);
        qzd = ((B[2][cj][ci] + B[2][cj][ci + 1]) + B[2][cj + 1][ci]) + B[2][cj + 1][ci + 1];
      }
      // work = sum_p S_cp . delta_p (= dt sum S.u_bar) of cell plane k-1
      const double work = (m.ax * (pxd + qxd) + m.ay * (pyd + qyd)) + m.az * (qzd - pzd);
      pxd = qxd;
      pyd = qyd;
      pzd = qzd;
      const bool mine = own_cell && cp >= Z0 && cp < Z1;
      double vx = 0.0, vy = 0.0, dvz_up = 0.0;
      // the cells whose lower x / y faces are formed: the owned ones, with RL
      // also the first halo column (x) and row (y) above them, whose lower
      // faces are the owned cells' upper faces (a wall face stays zero)
      const bool fx = RL ? plane_ok && ci >= 1 && ci <= TX + 1 && cj >= 1 && cj <= TY && gi <= m.nx - 1 && gj < m.ny
                         : mine && plane_ok;
      const bool fy = RL ? plane_ok && ci >= 1 && ci <= TX && cj >= 1 && cj <= TY + 1 && gi < m.nx && gj <= m.ny - 1
                         : mine && plane_ok;
      // lower x face (node column gi, between cells gi-1 and gi); corners (s: y, t: z)
      if (fx && gi >= 1) {
        const double d0[3] = {A[0][cj][ci], A[1][cj][ci], A[2][cj][ci]};
        const double d1[3] = {A[0][cj + 1][ci], A[1][cj + 1][ci], A[2][cj + 1][ci]};
        const double d2[3] = {B[0][cj][ci], B[1][cj][ci], B[2][cj][ci]};
        const double d3[3] = {B[0][cj + 1][ci], B[1][cj + 1][ci], B[2][cj + 1][ci]};
        vx = swept_volume(d0, d1, d2, d3, m.ax, m.edy, m.edz);
      }
      // lower y face (node row gj, between cells gj-1 and gj); corners (s: z, t: x); comps (y, z, x)
      if (fy && gj >= 1) {
        const double d0[3] = {A[1][cj][ci], A[2][cj][ci], A[0][cj][ci]};
        const double d1[3] = {B[1][cj][ci], B[2][cj][ci], B[0][cj][ci]};
        const double d2[3] = {A[1][cj][ci + 1], A[2][cj][ci + 1], A[0][cj][ci + 1]};
        const double d3[3] = {B[1][cj][ci + 1], B[2][cj][ci + 1], B[0][cj][ci + 1]};
        vy = swept_volume(d0, d1, d2, d3, m.ay, m.edz, m.edx);
      }
      // z face at node plane k between cells k-1 and k (the lower z face of
      // cell plane k); corners (s: x, t: y); comps (z, x, y)
      if (own_cell && k >= 1 && k <= m.nz - 1) {
        const double d0[3] = {B[2][cj][ci], B[0][cj][ci], B[1][cj][ci]};
        const double d1[3] = {B[2][cj][ci + 1], B[0][cj][ci + 1], B[1][cj][ci + 1]};
        const double d2[3] = {B[2][cj + 1][ci], B[0][cj + 1][ci], B[1][cj + 1][ci]};
        const double d3[3] = {B[2][cj + 1][ci + 1], B[0][cj + 1][ci + 1], B[1][cj + 1][ci + 1]};
        dvz_up = swept_volume(d0, d1, d2, d3, m.az, m.edx, m.edy);
      }
      if constexpr (RL) {  // FP64, whatever the bulk type of the hand-off
        sVX[cj][ci] = vx;
        sVY[cj][ci] = vy;
      }
      settle(fu), settle(fv), settle(fw), settle(frho), settle(fe);  // loads issued in P1
      if (mine) {
        const uint32_t oR = cix * (uint32_t)sizeof(R);
        plane_at<R>(a.geo.el, cpl, cp, oR) = R((double)e1 - (double)ps1 * work / (double)m1);
        plane_at<R>(a.geo.dvx, cpl, cp, oR) = R(vx);
        plane_at<R>(a.geo.dvy, cpl, cp, oR) = R(vy);
        plane_at<R>(a.geo.dvz, cpl, cp, oR) = R(dvz_lo);
      }
      if constexpr (RL) {
        // ---- P5: V^L and rho^L of cell plane k-1 ----
        __syncthreads();
        if (mine) {
          const double VL =
              m.V0 + (((sVX[cj][ci + 1] - sVX[cj][ci]) + (sVY[cj + 1][ci] - sVY[cj][ci])) + (dvz_up - dvz_lo));
          R rl = R(0);
          if (!(VL > 0.0))
            tangle = true;
          else
            rl = R((double)m1 / VL);
          plane_at<R>(a.geo.rl, cpl, cp, cix * (uint32_t)sizeof(R)) = rl;
        }
      }
      dvz_lo = dvz_up;
    }
    ps1 = ps;
    e1 = e_k;
    m1 = mc;
  }
  return tangle;
}

// ---------------------------------------------------------------------------------
// remap_tile: the Eulerian remap (O9..O11) and the next signal speed (O3)
// ---------------------------------------------------------------------------------
// Column (ci, cj) is node column / cell column (X0 + ci - 2, Y0 + cj - 2). The
// tile owns cells [X0, X0+TX) x [Y0, Y0+TY) of its z segment and the matching
// nodes (TX = 32, TY = CH - 4; halo two columns on each side). Iteration c:
//   P1  Lagrangian results of cell plane c+1 (halo 2 below, 1 above) and u'
//       of node plane c+1 into LDS (loaded one iteration earlier)
//   P2  donor-cell fluxes of the cell's lower and upper x/y faces (a face's
//       flux is formed by both of its cells, from the same operands, so
//       both get the same bits and no barrier is needed to share it) and of
//       the z face at node plane c+1; net x/y fluxes of plane c+1; M,
//       rho^{n+1}, e^pre of cell plane c
//   P4  dual fluxes (1/8 of the adjacent cells' face fluxes) and nodal masses
//       of node plane c
//   P5  momentum / kinetic-energy remap of node plane c: u^{n+1}, KE defect
//   P6  KE fix, e^{n+1} and signal speed of cell plane c-1
// u' is kept in a 3-plane LDS ring (node planes c-1, c, c+1).
// Writes the new state; returns the tile's largest signal speed in *amax and
// whether an owned cell or node was inadmissible in *bad.
template <typename R, int CH, int CW = kTileW, int NTH = tile_threads<CH>()>
__device__ void remap_tile(const RunArgs<R> &a, int b, double *lds, double *amax_out, bool *bad_out,
                           bool *tangle_out) {
  constexpr int TX = CW - 4, TY = CH - 4, CHL = lds_rows<CW, CH, NTH>();
  static_assert(CW * CH <= NTH, "one thread per column");
  const Mesh &m = a.m;
  int tx, ty, seg;
  tile_of(a.gb, b, tx, ty, seg);
  const int ci = threadIdx.x % CW, cj = threadIdx.x / CW;
  const int gi = tx * TX + ci - 2, gj = ty * TY + cj - 2;
  const int Z0 = seg * a.gb.seglen;
  const bool lastseg = seg == a.gb.nseg - 1;
  const int Z1 = lastseg ? m.nz : Z0 + a.gb.seglen;  // cell planes [Z0, Z1)
  const int NZ1 = lastseg ? m.nz + 1 : Z1;           // node planes [Z0, NZ1)
  const bool own_cell = ci >= 2 && cj >= 2 && ci < 2 + TX && cj < 2 + TY && gi < m.nx && gj < m.ny;
  const bool own_node = ci >= 2 && cj >= 2 && cj < CH && gi <= m.nx && gj <= m.ny && (ci < 2 + TX || gi == m.nx) &&
                        (cj < 2 + TY || gj == m.ny);

  // LDS: the x/y swept volumes of plane c+1 as double, then planes of R
  // (CW x (CH + 1) values each) reused across phases. P1 of the next plane writes
  // only RL, EL, the swept volumes and the u' ring, which P6 does not read,
  // so no barrier separates P6 from it; P2, which writes R planes 2..6, comes
  // after P1's barrier.
  enum {
    RL = 0, EL = 1,                          // Lagrangian results of plane c+1    (P1-P2)
    SX = 2, SY = 3, MM = 4, MO = 5, SZ = 6,  // flux and mass sums                (P2-P4)
    PHX = 0, PHY = 1,                        // dual fluxes of node plane c        (P4-P5)
    UN = 2, SP = 5, DK = 6,                  // 2..4 u^{n+1}; |u^{n+1}|; KE defect (P5-P6)
    NSLOT = 7
  };
  double(*sVX)[CW] = reinterpret_cast<double(*)[CW]>(lds);
  double(*sVY)[CW] = reinterpret_cast<double(*)[CW]>(lds + CHL * CW);
  R *const rbase = reinterpret_cast<R *>(lds + 2 * CHL * CW);
  auto RS = [&](int s) { return reinterpret_cast<R(*)[CW]>(rbase + s * CHL * CW); };
  R(*UPR)[3][CHL][CW] = reinterpret_cast<R(*)[3][CHL][CW]>(rbase + NSLOT * CHL * CW);  // [3][3]
  static_assert(2 * CHL * CW * 8 + (NSLOT + 9) * CHL * CW * (int)sizeof(R) <= remap_lds_doubles<R, CH, CW, NTH>() * 8,
                "remap LDS layout");

  const bool ccol = cj < CH && gi >= 0 && gi < m.nx && gj >= 0 && gj < m.ny;
  const bool ncol = cj < CH && gi >= 0 && gi <= m.nx && gj >= 0 && gj <= m.ny;
  const int64_t cpl = (int64_t)m.nx * m.ny, npl = (int64_t)(m.nx + 1) * (m.ny + 1);
  const uint32_t cix = ccol ? (uint32_t)(gi + m.nx * gj) : 0u, nix = ncol ? (uint32_t)(gi + (m.nx + 1) * gj) : 0u;
  const bool r1 = ci >= 1 && cj >= 1 && ci <= CW - 2 && cj <= CH - 2;  // cells and nodes [-1, T]
  const bool r2 = ci >= 2 && cj >= 2 && ci <= CW - 2 && cj <= CH - 2;  // nodes [0, T]
  const R V0 = R(m.V0), iV0 = R(m.iV0);

  // column carries: values of cell plane c / node plane c unless noted
  R rho_c = 0, rl_c = 0, el_c = 0;  // old density, rho^L, e^L
  R muz_c = 0, epz_c = 0;           // z-face fluxes at node plane c
  R nxm_c = 0, nxe_c = 0;           // x/y net outflows
  R ep_c1 = 0;                      // e^pre of cell plane c-1
  R qx_c = 0, qy_c = 0;             // 2-cell flux sums (dual x/y fluxes)
  R phx_c = 0, phy_c = 0;           // dual x/y fluxes of node plane c
  R phz_c1 = 0;                     // z dual flux between node planes c-1 and c
  R pm_c1 = 0, pr_c1 = 0;           // 4-cell sums of M and m of cell plane c-1
  R dks1 = 0, sm1 = 0, xn1 = 0, yn1 = 0, zn1 = 0;  // new-state partials of node plane c-1
  double amax = 0.0;
  bool bad = false;

  // global loads run one plane ahead
  // (cell plane cp: e^L, rho, the swept volumes of the cell's lower x and y
  // faces and of its upper x, y and z faces -- the lower faces of its +x,
  // +y and +z neighbours, zero on a wall)
  R f_el = 0, f_rho = 0, f_u = 0, f_v = 0, f_w = 0;
  R f_vx = 0, f_vy = 0, f_vxu = 0, f_vyu = 0, f_vzu = 0;
  const bool xup = ccol && gi + 1 < m.nx, yup = ccol && gj + 1 < m.ny;
  auto fetch = [&](int cp) {
    f_el = f_rho = f_u = f_v = f_w = R(0);
    f_vx = f_vy = f_vxu = f_vyu = f_vzu = R(0);
    if (ccol && cp >= 0 && cp < m.nz) {
      const uint32_t oR = cix * (uint32_t)sizeof(R);
      f_el = plane_at<const R>(a.geo.el, cpl, cp, oR);
      f_vx = plane_at<const R>(a.geo.dvx, cpl, cp, oR);
      f_vy = plane_at<const R>(a.geo.dvy, cpl, cp, oR);
      if (xup) f_vxu = plane_at<const R>(a.geo.dvx, cpl, cp, oR + (uint32_t)sizeof(R));
      if (yup) f_vyu = plane_at<const R>(a.geo.dvy, cpl, cp, oR + (uint32_t)(m.nx * sizeof(R)));
      if (cp + 1 < m.nz) f_vzu = plane_at<const R>(a.geo.dvz, cpl, cp + 1, oR);
      f_rho = plane_at<const R>(a.cur.rho, cpl, cp, oR);
    }
    // (u' is read by the momentum remap of nodes [2, CW-2] x [2, CH-2] from
    // their neighbours: column 0 and row 0 are never read)
    if (ncol && ci >= 1 && cj >= 1 && cp >= 0 && cp <= m.nz) {
      const uint32_t o = nix * (uint32_t)sizeof(R);
      f_u = plane_at<const R>(a.up, npl, cp, o);
      f_v = plane_at<const R>(a.vp, npl, cp, o);
      f_w = plane_at<const R>(a.wp, npl, cp, o);
    }
  };
  // the u' ring starts empty (node planes below Z0-2 only feed non-owned results)
  for (int q = threadIdx.x; q < 3 * 3 * CH * CW; q += NTH) (&UPR[0][0][0][0])[q] = R(0);
  fetch(Z0 - 2);
  // swept volume of the lower z face of cell plane c+1 (carried: the upper
  // face loaded with plane c)
  R dvz_n = 0;
  if (ccol && Z0 - 2 >= 1 && Z0 - 2 < m.nz) dvz_n = plane_at<const R>(a.geo.dvz, cpl, Z0 - 2, cix * (uint32_t)sizeof(R));
  settle(f_el), settle(f_rho), settle(f_u), settle(f_v), settle(f_w);
  settle(f_vx), settle(f_vy), settle(f_vxu), settle(f_vyu), settle(f_vzu), settle(dvz_n);
  bool tangle = false;
  __syncthreads();

  for (int c = Z0 - 3; c <= Z1; c++) {  // c >= -3
    const int c1 = c + 1;
    const int rA = (c + 5) % 3, rB = (c + 6) % 3, rC = (c + 7) % 3;  // ring rows of c-1, c, c+1
    // ---- P1 --------------------------------------------------------------------------
    const R el_n = f_el, rho_n = f_rho;
    // V^L and rho^L of cell plane c+1 from the swept volumes of its six faces
    R rl_n = 0;
    {
      const R mc = rho_n * V0;
      const double VL = m.V0 + ((((double)f_vxu - (double)f_vx) + ((double)f_vyu - (double)f_vy)) +
                                ((double)f_vzu - (double)dvz_n));
      if (ccol && c1 >= 0 && c1 < m.nz) {
        if (!(VL > 0.0)) {
          if (own_cell && c1 >= Z0 && c1 < Z1) tangle = true;
        } else {
          rl_n = R((double)mc / VL);
        }
      }
    }
    const double dvz_f = (double)dvz_n;  // z face between cell planes c and c+1
    dvz_n = f_vzu;
    RS(RL)[cj][ci] = rl_n;
    RS(EL)[cj][ci] = el_n;
    sVX[cj][ci] = (double)f_vx;
    sVY[cj][ci] = (double)f_vy;
    UPR[rC][0][cj][ci] = f_u;  // node plane c+1 (slot last read as plane c-2)
    UPR[rC][1][cj][ci] = f_v;
    UPR[rC][2][cj][ci] = f_w;
    fetch(c + 2);
    __syncthreads();
    const R uA = UPR[rA][0][cj][ci], vA = UPR[rA][1][cj][ci], wA = UPR[rA][2][cj][ci];
    const R uB = UPR[rB][0][cj][ci], vB = UPR[rB][1][cj][ci], wB = UPR[rB][2][cj][ci];
    const R uC = UPR[rC][0][cj][ci], vC = UPR[rC][1][cj][ci], wC = UPR[rC][2][cj][ci];
    // ---- P2 --------------------------------------------------------------------------
    R ep_c = 0;
    {
      const bool pl = c1 >= 0 && c1 < m.nz;
      // donor-cell fluxes through the x face at column x (between cells x-1
      // and x) and the y face at row y of plane c+1; zero on walls and
      // outside the mesh
      auto xflux = [&](int x, int gx, R &mu, R &ep) {
        mu = ep = R(0);
        if (pl && x >= 1 && gx >= 1 && gx <= m.nx - 1 && gj >= 0 && gj < m.ny) {
          const R dv = R(sVX[cj][x]);
          const int dn = sVX[cj][x] > 0.0 ? x - 1 : x;
          mu = RS(RL)[cj][dn] * dv;
          ep = mu * RS(EL)[cj][dn];
        }
      };
      auto yflux = [&](int y, int gy, R &mu, R &ep) {
        mu = ep = R(0);
        if (pl && y >= 1 && gy >= 1 && gy <= m.ny - 1 && gi >= 0 && gi < m.nx) {
          const R dv = R(sVY[y][ci]);
          const int dn = sVY[y][ci] > 0.0 ? y - 1 : y;
          mu = RS(RL)[dn][ci] * dv;
          ep = mu * RS(EL)[dn][ci];
        }
      };
      R muz_n = 0, epz_n = 0;
      if (ccol && c1 >= 1 && c1 <= m.nz - 1) {  // z face between cells c and c+1
        const bool lower = dvz_f > 0.0;
        muz_n = (lower ? rl_c : rl_n) * R(dvz_f);
        epz_n = muz_n * (lower ? el_c : el_n);
      }
      R nm = 0, ne = 0, sx = 0, sy = 0, M = 0, mo = 0, sz = 0;
      if (r1 && ccol && c1 >= 0 && c1 < m.nz) {
        R mxl, exl, mxu, exu, myl, eyl, myu, eyu;
        xflux(ci, gi, mxl, exl);
        xflux(ci + 1, gi + 1, mxu, exu);
        yflux(cj, gj, myl, eyl);
        yflux(cj + 1, gj + 1, myu, eyu);
        nm = (mxu - mxl) + (myu - myl);
        ne = (exu - exl) + (eyu - eyl);
        sx = mxl + mxu;
        sy = myl + myu;
      }
      if (r1 && ccol && c >= 0 && c < m.nz) {
        const R netm = nxm_c + (muz_n - muz_c);
        const R nete = nxe_c + (epz_n - epz_c);
        mo = rho_c * V0;
        M = mo - netm;
        const R rn = rho_c - netm * iV0;
        const bool mine = own_cell && c >= Z0 && c < Z1;
        if (!(M > R(0)) || !(rn > R(0)) || !isfinite(rn)) {
          if (mine) bad = true;
        } else {
          ep_c = el_c + (el_c * netm - nete) / M;
        }
        if (mine) plane_at<R>(a.nxt.rho, cpl, c, cix * (uint32_t)sizeof(R)) = rn;
        sz = muz_c + muz_n;
      }
      RS(SX)[cj][ci] = sx;  // slots the phase does not read
      RS(SY)[cj][ci] = sy;
      RS(MM)[cj][ci] = M;
      RS(MO)[cj][ci] = mo;
      RS(SZ)[cj][ci] = sz;
      nxm_c = nm;
      nxe_c = ne;
      // plane c+1 becomes plane c
      rho_c = rho_n;
      rl_c = rl_n;
      el_c = el_n;
      muz_c = muz_n;
      epz_c = epz_n;
    }
    __syncthreads();
    // ---- P4 --------------------------------------------------------------------------
    R phz = 0, mp = 0, mn = 0;
    {
      R qx = 0, qy = 0, pm = 0, pr = 0;
      if (r1) {
        const R(*SXs)[CW] = RS(SX);
        const R(*SYs)[CW] = RS(SY);
        const R(*SZs)[CW] = RS(SZ);
        const R(*MMs)[CW] = RS(MM);
        const R(*MOs)[CW] = RS(MO);
        qx = SXs[cj - 1][ci] + SXs[cj][ci];  // cells (i, j-1), (i, j) of plane c+1
        qy = SYs[cj][ci - 1] + SYs[cj][ci];
        phz = R(0.125) * (((SZs[cj - 1][ci - 1] + SZs[cj - 1][ci]) + SZs[cj][ci - 1]) + SZs[cj][ci]);
        pm = ((MMs[cj - 1][ci - 1] + MMs[cj - 1][ci]) + MMs[cj][ci - 1]) + MMs[cj][ci];
        pr = ((MOs[cj - 1][ci - 1] + MOs[cj - 1][ci]) + MOs[cj][ci - 1]) + MOs[cj][ci];
        mn = R(0.125) * (pm_c1 + pm);
        mp = R(0.125) * (pr_c1 + pr);
      }
      RS(PHX)[cj][ci] = phx_c;  // dual fluxes of node plane c (slots dead since P2)
      RS(PHY)[cj][ci] = phy_c;
      phx_c = R(0.125) * (qx_c + qx);  // node plane c+1
      phy_c = R(0.125) * (qy_c + qy);
      qx_c = qx;
      qy_c = qy;
      pm_c1 = pm;
      pr_c1 = pr;
    }
    __syncthreads();
    settle(f_el), settle(f_rho), settle(f_u), settle(f_v), settle(f_w);  // loads issued in P1
    settle(f_vx), settle(f_vy), settle(f_vxu), settle(f_vyu), settle(f_vzu);
    // ---- P5: node plane c --------------------------------------------------------------
    {
      R un = 0, vn = 0, wn = 0, sp = 0, dk = 0;
      if (r2 && ncol && c >= 0 && c <= m.nz) {
        R P0 = mp * uB, P1 = mp * vB, P2 = mp * wB;
        R K = R(0.5) * mp * (uB * uB + vB * vB + wB * wB);
        auto flow = [&](R phi, R ud, R vd, R wd, R sgn) {
          P0 += sgn * (phi * ud);
          P1 += sgn * (phi * vd);
          P2 += sgn * (phi * wd);
          K += sgn * (phi * R(0.5) * (ud * ud + vd * vd + wd * wd));
        };
        const R(*U)[CW] = UPR[rB][0];
        const R(*V)[CW] = UPR[rB][1];
        const R(*W)[CW] = UPR[rB][2];
        const R(*PX)[CW] = RS(PHX);
        const R(*PY)[CW] = RS(PHY);
        if (gi + 1 <= m.nx) {
          const R phi = PX[cj][ci];
          if (phi > R(0)) flow(phi, uB, vB, wB, R(-1));
          else flow(phi, U[cj][ci + 1], V[cj][ci + 1], W[cj][ci + 1], R(-1));
        }
        if (gi - 1 >= 0) {
          const R phi = PX[cj][ci - 1];
          if (phi > R(0)) flow(phi, U[cj][ci - 1], V[cj][ci - 1], W[cj][ci - 1], R(1));
          else flow(phi, uB, vB, wB, R(1));
        }
        if (gj + 1 <= m.ny) {
          const R phi = PY[cj][ci];
          if (phi > R(0)) flow(phi, uB, vB, wB, R(-1));
          else flow(phi, U[cj + 1][ci], V[cj + 1][ci], W[cj + 1][ci], R(-1));
        }
        if (gj - 1 >= 0) {
          const R phi = PY[cj - 1][ci];
          if (phi > R(0)) flow(phi, U[cj - 1][ci], V[cj - 1][ci], W[cj - 1][ci], R(1));
          else flow(phi, uB, vB, wB, R(1));
        }
        if (c + 1 <= m.nz) {
          const R phi = phz;
          if (phi > R(0)) flow(phi, uB, vB, wB, R(-1));
          else flow(phi, uC, vC, wC, R(-1));
        }
        if (c - 1 >= 0) {
          const R phi = phz_c1;
          if (phi > R(0)) flow(phi, uA, vA, wA, R(1));
          else flow(phi, uB, vB, wB, R(1));
        }
        const bool mine = own_node && c >= Z0 && c < NZ1;
        if (!(mn > R(0))) {
          if (mine) bad = true;
        } else {
          const R imn = R(1) / mn;
          un = P0 * imn;
          vn = P1 * imn;
          wn = P2 * imn;
          if (gi == 0 || gi == m.nx) un = R(0);
          if (gj == 0 || gj == m.ny) vn = R(0);
          if (c == 0 || c == m.nz) wn = R(0);
          dk = (K - R(0.5) * mn * (un * un + vn * vn + wn * wn)) * imn;
          sp = speed(un, vn, wn);
        }
        if (mine) {
          const uint32_t o = nix * (uint32_t)sizeof(R);
          plane_at<R>(a.nxt.u, npl, c, o) = un;
          plane_at<R>(a.nxt.v, npl, c, o) = vn;
          plane_at<R>(a.nxt.w, npl, c, o) = wn;
        }
      }
      RS(UN)[cj][ci] = un;
      RS(UN + 1)[cj][ci] = vn;
      RS(UN + 2)[cj][ci] = wn;
      RS(SP)[cj][ci] = sp;
      RS(DK)[cj][ci] = dk;
      phz_c1 = phz;
    }
    __syncthreads();
    // ---- P6: cell plane c-1 ------------------------------------------------------------
    {
      R dks = 0, sm = 0, xn = 0, yn = 0, zn = 0;
      if (r2 && ci <= CW - 3 && cj <= CH - 3) {
        const R(*U)[CW] = RS(UN);
        const R(*V)[CW] = RS(UN + 1);
        const R(*W)[CW] = RS(UN + 2);
        const R(*S)[CW] = RS(SP);
        const R(*Q)[CW] = RS(DK);
        dks = ((Q[cj][ci] + Q[cj][ci + 1]) + Q[cj + 1][ci]) + Q[cj + 1][ci + 1];
        sm = fmax(fmax(S[cj][ci], S[cj][ci + 1]), fmax(S[cj + 1][ci], S[cj + 1][ci + 1]));
        xn = (U[cj][ci + 1] - U[cj][ci]) + (U[cj + 1][ci + 1] - U[cj + 1][ci]);
        yn = (V[cj + 1][ci] - V[cj][ci]) + (V[cj + 1][ci + 1] - V[cj][ci + 1]);
        zn = ((W[cj][ci] + W[cj][ci + 1]) + W[cj + 1][ci]) + W[cj + 1][ci + 1];
        const int cm = c - 1;
        if (own_cell && cm >= Z0 && cm < Z1) {
          const R en = ep_c1 + R(0.125) * (dks1 + dks);
          plane_at<R>(a.nxt.e, cpl, cm, cix * (uint32_t)sizeof(R)) = en;
          const R D = divergence(m, xn1, xn, yn1, yn, zn1, zn);
          const R sa = signal_from(m, D, en, fmax(sm1, sm));
          if (!(en >= R(0)) || !isfinite(en) || !isfinite(sa))
            bad = true;
          else
            amax = fmax(amax, (double)sa);
        }
      }
      dks1 = dks;
      sm1 = sm;
      xn1 = xn;
      yn1 = yn;
      zn1 = zn;
      ep_c1 = ep_c;
    }
  }
  __syncthreads();  // the last plane's P6 reads are done before the LDS is reused
  *amax_out = amax;
  *bad_out = bad;
  *tangle_out = tangle;
}

// No-op step of a tile: carry the owned part of the state into the other buffer.
template <typename R, int CH>
__device__ void copy_tile(const RunArgs<R> &a, int b) {
  constexpr int CW = kTileW, TX = CW - 4, TY = CH - 4;
  const Mesh &m = a.m;
  int tx, ty, seg;
  tile_of(a.gb, b, tx, ty, seg);
  const int ci = threadIdx.x % CW, cj = threadIdx.x / CW;
  const int gi = tx * TX + ci - 2, gj = ty * TY + cj - 2;
  const int Z0 = seg * a.gb.seglen;
  const bool lastseg = seg == a.gb.nseg - 1;
  const int Z1 = lastseg ? m.nz : Z0 + a.gb.seglen;
  const int NZ1 = lastseg ? m.nz + 1 : Z1;
  const bool own_cell = ci >= 2 && cj >= 2 && ci < 2 + TX && cj < 2 + TY && gi < m.nx && gj < m.ny;
  const bool own_node = ci >= 2 && cj >= 2 && cj < CH && gi <= m.nx && gj <= m.ny && (ci < 2 + TX || gi == m.nx) &&
                        (cj < 2 + TY || gj == m.ny);
  for (int c = Z0; c < Z1; c++)
    if (own_cell) {
      const int64_t q = cidx(m, gi, gj, c);
      a.nxt.rho[q] = a.cur.rho[q];
      a.nxt.e[q] = a.cur.e[q];
    }
  for (int n = Z0; n < NZ1; n++)
    if (own_node) {
      const int64_t q = nidx(m, gi, gj, n);
      a.nxt.u[q] = a.cur.u[q];
      a.nxt.v[q] = a.cur.v[q];
      a.nxt.w[q] = a.cur.w[q];
    }
}

}  // namespace sale
