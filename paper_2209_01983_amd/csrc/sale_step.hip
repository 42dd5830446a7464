// sale_step.hip -- single-run kernels of libsale for gfx950: the step
// (k_begin, k_lagrange, k_remap around the tile functions of sale_tiles.h),
// initial states, diagnostics, field export and the workspace layout, for
// both precisions (R = double: SALE_FP64, R = float: SALE_MIXED32).
#include "sale_tiles.h"

namespace sale {
namespace {

// The two z-marching kernels are templates on their tile rows CH (tiles of
// kTileW x CH columns, one thread each, in blocks of tile_threads<CH>()); the
// launch shape picks CH per kernel at run time: 7, 14 or 28 rows (256, 512,
// 1024 threads). Each shape has a register cap (minimum waves per SIMD): a
// block of 512 threads puts 2 waves on each SIMD, so the cap fixes how many
// blocks share a CU. Register spills are to be avoided: their reloads wait
// for every outstanding global load and store of the wave.
#ifndef SALE_WAVES_14
#define SALE_WAVES_14 4
#endif
template <int CH>
constexpr int waves_of() {
  return CH == 14 ? SALE_WAVES_14 : 4;
}
// The FP32 bulk remap tile of 14 rows fits 80 VGPRs and its LDS (bulk planes
// as float) 42 KB: three blocks per CU.
// (The FP64 remap tile of 7 rows needs 41 KB of LDS: three blocks per CU.)
template <typename R, int CH>
constexpr int remap_waves() {
  return sizeof(R) == 4 && CH == 14 ? 6 : sizeof(R) == 8 && CH == 7 ? 3 : waves_of<CH>();
}
constexpr int TPB = 256;  // simple per-element kernels

// ---------------------------------------------------------------------------------
// k_begin: the step's time step (O3) and the done decision
// ---------------------------------------------------------------------------------
__global__ void k_begin(Mesh m, Ctl *ctl) {
  if (threadIdx.x == 0 && blockIdx.x == 0) begin_step(m, ctl, 0x7fffffffffffffffll);
}

// (RL: the second-order step's Lagrange kernel, which also forms rho^L)
template <typename R, int CH, bool RL = false>
__global__ __launch_bounds__(tile_threads<CH>(), waves_of<CH>()) void k_lagrange(RunArgs<R> a) {
  __shared__ double lds[lagrange_lds_doubles<CH, kTileWL, tile_threads<CH>(), RL>()];
  if (a.ctl->done) return;
  const bool t =
      lagrange_tile<R, CH, kTileWL, tile_threads<CH>(), RL>(a, xcd_logical_block(blockIdx.x, gridDim.x), a.ctl->dt, lds);
  if (t) atomicOr(&a.ctl->status, SALE_FLAG_TANGLE);
}

template <typename R, int CH>
__global__ __launch_bounds__(tile_threads<CH>(), (remap_waves<R, CH>())) void k_remap(RunArgs<R> a) {
  __shared__ double lds[remap_lds_doubles<R, CH>()];
  const int b = xcd_logical_block(blockIdx.x, gridDim.x);
  if (a.ctl->done) {
    copy_tile<R, CH>(a, b);
    return;
  }
  double amax;
  bool bad, tangle;
  remap_tile<R, CH>(a, b, lds, &amax, &bad, &tangle);
  block_max_to_ctl<tile_threads<CH>()>(a.ctl, amax, bad);
  if (tangle) atomicOr(&a.ctl->status, SALE_FLAG_TANGLE);
}

// ---------------------------------------------------------------------------------
// initial states, signal speed of a state, diagnostics, export
// ---------------------------------------------------------------------------------
__device__ __forceinline__ void cell_ijk(const Mesh &m, int64_t c, int &i, int &j, int &k) {
  i = (int)(c % m.nx);
  const int64_t r = c / m.nx;
  j = (int)(r % m.ny);
  k = (int)(r / m.ny);
}
__device__ __forceinline__ void node_ijk(const Mesh &m, int64_t n, int &i, int &j, int &k) {
  i = (int)(n % (m.nx + 1));
  const int64_t r = n / (m.nx + 1);
  j = (int)(r % (m.ny + 1));
  k = (int)(r / (m.ny + 1));
}

template <typename R>
__global__ __launch_bounds__(TPB) void k_signal(Mesh m, Ctl *ctl, State<R> s) {
  const int64_t c = blockIdx.x * (int64_t)TPB + threadIdx.x;
  double a = 0.0;
  bool bad = false;
  if (c < m.ncell) {
    int i, j, k;
    cell_ijk(m, c, i, j, k);
    const R D = state_divergence(m, s, i, j, k);
    R smax = 0;
    for (int cc = 0; cc < 2; cc++)
      for (int b = 0; b < 2; b++)
        for (int aa = 0; aa < 2; aa++) {
          const int64_t n = nidx(m, i + aa, j + b, k + cc);
          const R sp = speed(s.u[n], s.v[n], s.w[n]);
          if (!isfinite(sp)) bad = true;
          smax = fmax(smax, sp);
        }
    const R rho = s.rho[c], e = s.e[c];
    const R sa = signal_from(m, D, e, smax);
    a = (double)sa;
    if (!(rho > R(0)) || !isfinite(rho) || !(e >= R(0)) || !isfinite(e) || !isfinite(sa)) bad = true;
  }
  block_max_to_ctl<TPB>(ctl, a, bad);
}

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
  ctl->tiles_done = 0u;
  ctl->phase = 0u;
  ctl->step_target = 0;
  ctl->clk_first = 0;
  ctl->clk_last = 0;
}

__global__ void k_set_t_end(Ctl *ctl, double t_end) {
  if (threadIdx.x == 0 && blockIdx.x == 0) ctl->t_end = t_end;
}

template <typename R>
__global__ __launch_bounds__(TPB) void k_init_cells_sod(Mesh m, State<R> s, double xs, double rL, double pL,
                                                       double rR, double pR) {
  const int64_t c = blockIdx.x * (int64_t)TPB + threadIdx.x;
  if (c >= m.ncell) return;
  int i, j, k;
  cell_ijk(m, c, i, j, k);
  const double xc = m.lo[0] + (i + 0.5) * m.dx;
  const bool left = xc < xs;
  const double r = left ? rL : rR;
  s.rho[c] = R(r);
  s.e[c] = R((left ? pL : pR) / ((m.gamma - 1.0) * r));
}

template <typename R>
__global__ __launch_bounds__(TPB) void k_init_cells_sedov(Mesh m, State<R> s, double r0, double p0,
                                                         double edep) {
  const int64_t c = blockIdx.x * (int64_t)TPB + threadIdx.x;
  if (c >= m.ncell) return;
  s.rho[c] = R(r0);
  s.e[c] = R(c == 0 ? edep / (r0 * m.V0) : p0 / ((m.gamma - 1.0) * r0));
}

// Noh: uniform cells; node velocity -u0 r/|r| toward the corner lo over the
// first `dims` axes, wall-normal components zeroed. Products are rounded on
// their own (not fused into the sums), as the definition is written.
template <typename R>
__global__ __launch_bounds__(TPB) void k_init_cells_uniform(Mesh m, State<R> s, double r0, double p0) {
  const int64_t c = blockIdx.x * (int64_t)TPB + threadIdx.x;
  if (c >= m.ncell) return;
  s.rho[c] = R(r0);
  s.e[c] = R(p0 / ((m.gamma - 1.0) * r0));
}

template <typename R>
__global__ __launch_bounds__(TPB) void k_init_nodes_noh(Mesh m, State<R> s, double u0, int dims) {
  const int64_t n = blockIdx.x * (int64_t)TPB + threadIdx.x;
  if (n >= m.nnode) return;
  int i, j, k;
  node_ijk(m, n, i, j, k);
  const double r[3] = {mul_rn(i, m.dx), dims >= 2 ? mul_rn(j, m.dy) : 0.0, dims >= 3 ? mul_rn(k, m.dz) : 0.0};
  const double len = sqrt((mul_rn(r[0], r[0]) + mul_rn(r[1], r[1])) + mul_rn(r[2], r[2]));
  double vel[3] = {0.0, 0.0, 0.0};
  if (len > 0.0)
    for (int a = 0; a < 3; a++) vel[a] = -u0 * (r[a] / len);
  if (i == 0 || i == m.nx) vel[0] = 0.0;
  if (j == 0 || j == m.ny) vel[1] = 0.0;
  if (k == 0 || k == m.nz) vel[2] = 0.0;
  s.u[n] = R(vel[0]);
  s.v[n] = R(vel[1]);
  s.w[n] = R(vel[2]);
}

template <typename R>
__global__ __launch_bounds__(TPB) void k_zero_nodes(Mesh m, State<R> s) {
  const int64_t n = blockIdx.x * (int64_t)TPB + threadIdx.x;
  if (n >= m.nnode) return;
  s.u[n] = s.v[n] = s.w[n] = R(0);
}

// copy a double array into an R array (user initial data)
template <typename R>
__global__ __launch_bounds__(TPB) void k_from_double(const double *src, R *dst, int64_t n) {
  const int64_t q = blockIdx.x * (int64_t)TPB + threadIdx.x;
  if (q < n) dst[q] = R(src[q]);
}

template <typename R>
__global__ __launch_bounds__(TPB) void k_wall_normals(Mesh m, State<R> s) {
  const int64_t n = blockIdx.x * (int64_t)TPB + threadIdx.x;
  if (n >= m.nnode) return;
  int i, j, k;
  node_ijk(m, n, i, j, k);
  if (i == 0 || i == m.nx) s.u[n] = R(0);
  if (j == 0 || j == m.ny) s.v[n] = R(0);
  if (k == 0 || k == m.nz) s.w[n] = R(0);
}

constexpr int TOT_BLOCKS = 1024;

template <typename R>
__global__ __launch_bounds__(TPB) void k_totals_partial(Mesh m, State<R> s, double *partial) {
  double sm = 0.0, si = 0.0, sk = 0.0;
  for (int64_t c = blockIdx.x * (int64_t)TPB + threadIdx.x; c < m.ncell; c += (int64_t)TOT_BLOCKS * TPB) {
    const double mc = (double)s.rho[c] * m.V0;
    sm += mc;
    si += mc * (double)s.e[c];
  }
  for (int64_t n = blockIdx.x * (int64_t)TPB + threadIdx.x; n < m.nnode; n += (int64_t)TOT_BLOCKS * TPB) {
    int i, j, k;
    node_ijk(m, n, i, j, k);
    double ms = 0.0;
    for (int cc = -1; cc <= 0; cc++)
      for (int b = -1; b <= 0; b++)
        for (int a = -1; a <= 0; a++)
          if (cell_in(m, i + a, j + b, k + cc)) ms += (double)s.rho[cidx(m, i + a, j + b, k + cc)] * m.V0;
    const double u = s.u[n], v = s.v[n], w = s.w[n];
    sk += 0.5 * (0.125 * ms) * (u * u + v * v + w * w);
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
    partial[threadIdx.x * TOT_BLOCKS + blockIdx.x] = r;
  }
}

// pure-Lagrangian mode: cell masses are stored (constant), not rho V0
__global__ __launch_bounds__(TPB) void k_lag_totals_partial(Mesh m, State<double> s, const double *mass,
                                                            double *partial) {
  double sm = 0.0, si = 0.0, sk = 0.0;
  for (int64_t c = blockIdx.x * (int64_t)TPB + threadIdx.x; c < m.ncell; c += (int64_t)TOT_BLOCKS * TPB) {
    sm += mass[c];
    si += mass[c] * s.e[c];
  }
  for (int64_t n = blockIdx.x * (int64_t)TPB + threadIdx.x; n < m.nnode; n += (int64_t)TOT_BLOCKS * TPB) {
    int i, j, k;
    node_ijk(m, n, i, j, k);
    double ms = 0.0;
    for (int cc = -1; cc <= 0; cc++)
      for (int b = -1; b <= 0; b++)
        for (int a = -1; a <= 0; a++)
          if (cell_in(m, i + a, j + b, k + cc)) ms += mass[cidx(m, i + a, j + b, k + cc)];
    const double u = s.u[n], v = s.v[n], w = s.w[n];
    sk += 0.5 * (0.125 * ms) * (u * u + v * v + w * w);
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
    partial[threadIdx.x * TOT_BLOCKS + blockIdx.x] = r;
  }
}

__global__ __launch_bounds__(TPB) void k_totals_final(Ctl *ctl, const double *partial) {
  __shared__ double red[3][TPB / 64];
  double s[3];
  for (int a = 0; a < 3; a++) {
    double x = 0.0;
    for (int b = threadIdx.x; b < TOT_BLOCKS; b += TPB) x += partial[a * TOT_BLOCKS + b];
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

// field `which` as double: 0 rho, 1 e, 2 p, 3 q, 4 u, 5 v, 6 w
template <typename R>
__global__ __launch_bounds__(TPB) void k_export(Mesh m, State<R> s, int which, double *out) {
  const int64_t q = blockIdx.x * (int64_t)TPB + threadIdx.x;
  if (which >= 4) {
    if (q >= m.nnode) return;
    const R *src = which == 4 ? s.u : (which == 5 ? s.v : s.w);
    out[q] = (double)src[q];
    return;
  }
  if (q >= m.ncell) return;
  const R rho = s.rho[q], e = s.e[q];
  if (which == 0) {
    out[q] = (double)rho;
  } else if (which == 1) {
    out[q] = (double)e;
  } else if (which == 2) {
    out[q] = (double)((R(m.gamma) - R(1)) * rho * e);
  } else {
    int i, j, k;
    cell_ijk(m, q, i, j, k);
    const R gm = R(m.gamma), h = R(m.h);
    const R cs = sqrt(gm * (gm - R(1)) * fmax(e, R(0)));
    const R D = state_divergence(m, s, i, j, k);
    R qv = 0;
    if (D < R(0)) {
      const R hd = h * D;
      qv = rho * (R(m.cq) * hd * hd + R(m.cl) * cs * h * fabs(D));
    }
    out[q] = (double)qv;
  }
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + TPB - 1) / TPB); }

// z segments so that tiles x segments fills the chip a few times over
// Split of the z extent into segments. A block marches its segment plus
// `warm` warm-up planes. target_blocks > 0: aim at that many blocks, with at
// least 8 planes per segment. target_blocks == 0 (automatic): a mesh whose
// blocks, at 8 planes per segment, all fit on the chip at once (`resident`)
// is latency bound -- split it as finely as keeps the fewest block rounds
// times the planes each block marches; a larger mesh aims at 3072 blocks.
Grid2 make_grid(int nx, int ny, int nplanes, int tile_x, int tile_y, int target_blocks, int warm, int resident) {
  Grid2 g;
  g.tx = (nx + tile_x - 1) / tile_x;
  g.ty = (ny + tile_y - 1) / tile_y;
  const int tiles = g.tx * g.ty;
  const int maxseg = nplanes / 8 > 1 ? nplanes / 8 : 1;  // >= 8 planes per segment
  int nseg;
  if (target_blocks == 0 && (long long)tiles * maxseg <= resident) {
    nseg = 1;
    long long best = -1;
    for (int s = 1; s <= nplanes; s++) {
      const long long rounds = ((long long)tiles * s + resident - 1) / resident;
      const long long cost = rounds * ((nplanes + s - 1) / s + warm);
      if (best < 0 || cost < best) {
        best = cost;
        nseg = s;
      }
    }
  } else {
    const int target = target_blocks > 0 ? target_blocks : 3072;
    nseg = (target + tiles / 2) / tiles;
    if (nseg > maxseg) nseg = maxseg;
    if (nseg < 1) nseg = 1;
  }
  g.seglen = (nplanes + nseg - 1) / nseg;
  g.nseg = (nplanes + g.seglen - 1) / g.seglen;
  return g;
}

}  // namespace

// blocks of a step kernel resident on MI355X at once (256 CUs), by tile rows
static int resident_blocks(int rows) {
  switch (rows) {
    case 7: return 4 * 256;
    case 14: return 2 * 256;
    default: return 256;
  }
}
Grid2 grid_lagrange(const Mesh &m, int target_blocks, int rows, int width) {
  return make_grid(m.nx, m.ny, m.nz, width - 3, rows - 3, target_blocks, 3, resident_blocks(rows));
}
Grid2 grid_remap(const Mesh &m, int target_blocks, int rows, int width) {
  return make_grid(m.nx, m.ny, m.nz, width - 4, rows - 4, target_blocks, 4, resident_blocks(rows));
}

bool launch_valid(const Launch &L) {
  auto ok = [](int r) { return r == 7 || r == 14 || r == 28; };
  return ok(L.rows_a) && ok(L.rows_b) && L.target >= 0 && L.target <= (1 << 20);
}

// ---- workspace layout -----------------------------------------------------------------
static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// The workspace is two parts: the state part (control block and the two
// state buffers) and the intermediates (u', the Lagrangian cell results,
// reduction partials, the scratch array, and the second-order and
// pure-Lagrangian arrays). A single-run workspace holds both back to back;
// sale_init_static puts the intermediates in the library's device array.
// Every array is followed by a gap of 33 blocks of 256 bytes, so that arrays
// of a power-of-two size do not start at one offset modulo that size (the
// streams a kernel reads side by side would meet in the same memory
// channels). At 320^3 in FP64 the gap is worth 1% of the step (gaps of 1 to
// 129 blocks measure the same).
constexpr size_t kGap = 33 * 256;

template <typename R>
size_t state_bytes(const Mesh &m) {
  const size_t cR = align256((size_t)m.ncell * sizeof(R)), nR = align256((size_t)m.nnode * sizeof(R));
  return align256(sizeof(Ctl)) + 2 * (2 * cR + 3 * nR) + 10 * kGap;
}

template <typename R>
size_t inter_bytes(const Mesh &m) {
  const size_t cR = align256((size_t)m.ncell * sizeof(R)), nR = align256((size_t)m.nnode * sizeof(R));
  const size_t sD = align256((size_t)(m.ncell > m.nnode ? m.ncell : m.nnode) * sizeof(double));
  // u' | e^L | 3 swept volumes | partials | scratch
  // (+ rho^L and the second-order remap's intermediates for order 2)
  const size_t r2 = m.order == 2 ? 6 * cR + nR : 0;
  const size_t cD = align256((size_t)m.ncell * sizeof(double)), nD = align256((size_t)m.nnode * sizeof(double));
  // positions x2, masses, corner forces
  const size_t lg = m.mode == 1 ? 6 * nD + cD + align256(24 * (size_t)corner_stride(m.ncell) * sizeof(double)) : 0;
  const size_t arrays = 9 + (m.order == 2 ? 7 : 0) + (m.mode == 1 ? 8 : 0);
  return 3 * nR + cR + 3 * cR + align256(3 * TOT_BLOCKS * sizeof(double)) + sD + r2 + lg + arrays * kGap;
}

template <typename R>
size_t workspace_bytes(const Mesh &m) {
  return state_bytes<R>(m) + inter_bytes<R>(m);
}

template <typename R>
void layout_split(const Mesh &m, void *state, void *inter, Ctl **ctl, Work<R> *w) {
  const size_t cR = align256((size_t)m.ncell * sizeof(R)), nR = align256((size_t)m.nnode * sizeof(R));
  const size_t sD = align256((size_t)(m.ncell > m.nnode ? m.ncell : m.nnode) * sizeof(double));
  char *p = (char *)state;
  *ctl = (Ctl *)p;
  p += align256(sizeof(Ctl));
  auto takeR = [&](size_t b) {
    R *r = (R *)p;
    p += b + kGap;
    return r;
  };
  auto takeD = [&](size_t b) {
    double *r = (double *)p;
    p += b + kGap;
    return r;
  };
  for (int a = 0; a < 2; a++) {
    w->s[a].rho = takeR(cR);
    w->s[a].e = takeR(cR);
    w->s[a].u = takeR(nR);
    w->s[a].v = takeR(nR);
    w->s[a].w = takeR(nR);
  }
  p = (char *)inter;
  w->geo.rl = nullptr;
  w->up = takeR(nR);
  w->vp = takeR(nR);
  w->wp = takeR(nR);
  w->geo.el = takeR(cR);
  w->geo.dvx = takeR(cR);
  w->geo.dvy = takeR(cR);
  w->geo.dvz = takeR(cR);
  w->partial = takeD(align256(3 * TOT_BLOCKS * sizeof(double)));
  w->scratch = takeD(sD);
  w->r2 = Rem2<R>{};
  if (m.order == 2) {
    w->geo.rl = takeR(cR);
    for (int a = 0; a < 3; a++) w->r2.mu[a] = takeR(cR);
    w->r2.M = takeR(cR);
    w->r2.epre = takeR(cR);
    w->r2.dk = takeR(nR);
  }
  w->lg = Lag{};
  if (m.mode == 1) {
    const size_t cD = align256((size_t)m.ncell * sizeof(double)), nD = align256((size_t)m.nnode * sizeof(double));
    for (int a = 0; a < 2; a++) {
      w->lg.x[a] = takeD(nD);
      w->lg.y[a] = takeD(nD);
      w->lg.z[a] = takeD(nD);
    }
    w->lg.m = takeD(cD);
    w->lg.F = takeD(align256(24 * (size_t)corner_stride(m.ncell) * sizeof(double)));
  }
}

template <typename R>
void layout(const Mesh &m, void *ws, Ctl **ctl, Work<R> *w) {
  layout_split<R>(m, ws, (char *)ws + state_bytes<R>(m), ctl, w);
}

// ---- launchers ----------------------------------------------------------------------------
template <typename R>
static hipError_t finish_init(const Mesh &m, Ctl *ctl, const Work<R> &w, double t0, long long step0,
                              double t_end, hipStream_t s) {
  hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, s, ctl, t0, step0, t_end);
  hipLaunchKernelGGL(k_signal<R>, dim3(blocks(m.ncell)), dim3(TPB), 0, s, m, ctl, w.s[0]);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_init_sod(const Mesh &m, Ctl *ctl, const Work<R> &w, const double sod[5], double t0,
                           long long step0, double t_end, hipStream_t s) {
  hipLaunchKernelGGL(k_init_cells_sod<R>, dim3(blocks(m.ncell)), dim3(TPB), 0, s, m, w.s[0], sod[0], sod[1],
                     sod[2], sod[3], sod[4]);
  hipLaunchKernelGGL(k_zero_nodes<R>, dim3(blocks(m.nnode)), dim3(TPB), 0, s, m, w.s[0]);
  return finish_init(m, ctl, w, t0, step0, t_end, s);
}

template <typename R>
hipError_t launch_init_sedov(const Mesh &m, Ctl *ctl, const Work<R> &w, const double sedov[3], double t0,
                             long long step0, double t_end, hipStream_t s) {
  hipLaunchKernelGGL(k_init_cells_sedov<R>, dim3(blocks(m.ncell)), dim3(TPB), 0, s, m, w.s[0], sedov[0],
                     sedov[1], sedov[2]);
  hipLaunchKernelGGL(k_zero_nodes<R>, dim3(blocks(m.nnode)), dim3(TPB), 0, s, m, w.s[0]);
  return finish_init(m, ctl, w, t0, step0, t_end, s);
}

template <typename R>
hipError_t launch_init_noh(const Mesh &m, Ctl *ctl, const Work<R> &w, const double noh[3], int dims, double t0,
                           long long step0, double t_end, hipStream_t s) {
  hipLaunchKernelGGL(k_init_cells_uniform<R>, dim3(blocks(m.ncell)), dim3(TPB), 0, s, m, w.s[0], noh[0], noh[1]);
  hipLaunchKernelGGL(k_init_nodes_noh<R>, dim3(blocks(m.nnode)), dim3(TPB), 0, s, m, w.s[0], noh[2], dims);
  return finish_init(m, ctl, w, t0, step0, t_end, s);
}

template <typename R>
hipError_t launch_init_user(const Mesh &m, Ctl *ctl, const Work<R> &w, const double *const src[5],
                            bool on_device, double t0, long long step0, double t_end, hipStream_t s) {
  R *dst[5] = {w.s[0].rho, w.s[0].e, w.s[0].u, w.s[0].v, w.s[0].w};
  for (int a = 0; a < 5; a++) {
    const int64_t n = a < 2 ? m.ncell : m.nnode;
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    hipError_t e = hipMemcpyAsync(w.scratch, src[a], (size_t)n * sizeof(double), kind, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_from_double<R>, dim3(blocks(n)), dim3(TPB), 0, s, (const double *)w.scratch, dst[a], n);
    // a host source must not be touched after return, and the scratch array
    // is reused by the next field: host copies wait here
    if (!on_device && (e = hipStreamSynchronize(s)) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_wall_normals<R>, dim3(blocks(m.nnode)), dim3(TPB), 0, s, m, w.s[0]);
  return finish_init(m, ctl, w, t0, step0, t_end, s);
}

hipError_t launch_set_t_end(Ctl *ctl, double t_end, hipStream_t s) {
  hipLaunchKernelGGL(k_set_t_end, dim3(1), dim3(64), 0, s, ctl, t_end);
  return hipGetLastError();
}

template <typename R>
RunArgs<R> run_args(const Mesh &m, Ctl *ctl, const Work<R> &w, int cur, const Launch &L) {
  RunArgs<R> a;
  a.m = m;
  a.ctl = ctl;
  a.cur = w.s[cur];
  a.nxt = w.s[1 - cur];
  a.up = w.up;
  a.vp = w.vp;
  a.wp = w.wp;
  a.geo = w.geo;
  a.ga = grid_lagrange(m, L.target, L.rows_a, kTileWL);
  a.gb = grid_remap(m, L.target, L.rows_b, kTileW);
  return a;
}

template <typename R, int CH>
void launch_lagrange(const RunArgs<R> &a, hipStream_t s) {
  if (a.m.order == 2)  // the second-order remap's passes take rho^L from the Lagrange kernel
    hipLaunchKernelGGL((k_lagrange<R, CH, true>), dim3(a.ga.blocks()), dim3(tile_threads<CH>()), 0, s, a);
  else
    hipLaunchKernelGGL((k_lagrange<R, CH>), dim3(a.ga.blocks()), dim3(tile_threads<CH>()), 0, s, a);
}
template <typename R, int CH>
void launch_remap(const RunArgs<R> &a, hipStream_t s) {
  hipLaunchKernelGGL((k_remap<R, CH>), dim3(a.gb.blocks()), dim3(tile_threads<CH>()), 0, s, a);
}

template <typename R>
hipError_t launch_step(const Mesh &m, Ctl *ctl, const Work<R> &w, int cur, const Launch &L, hipStream_t s,
                       const hipEvent_t *ev) {
  if (!launch_valid(L)) return hipErrorInvalidValue;
  if (m.mode == 1) {  // pure Lagrangian (FP64 only; the API refuses other precisions)
    if constexpr (std::is_same<R, double>::value)
      return launch_lag_step(m, ctl, w, cur, s, ev);
    else
      return hipErrorInvalidValue;
  }
  const RunArgs<R> a = run_args<R>(m, ctl, w, cur, L);
  hipError_t e = hipSuccess;
  if (ev) e = hipEventRecord(ev[0], s);
  hipLaunchKernelGGL(k_begin, dim3(1), dim3(64), 0, s, m, ctl);
  if (ev && e == hipSuccess) e = hipEventRecord(ev[1], s);
  switch (L.rows_a) {
    case 7: launch_lagrange<R, 7>(a, s); break;
    case 28: launch_lagrange<R, 28>(a, s); break;
    default: launch_lagrange<R, 14>(a, s); break;
  }
  if (ev && e == hipSuccess) e = hipEventRecord(ev[2], s);
  if (m.order == 2) {
    const hipError_t r = launch_remap2<R>(m, ctl, w, cur, s);
    if (r != hipSuccess) return r;
  } else {
    switch (L.rows_b) {
      case 7: launch_remap<R, 7>(a, s); break;
      case 28: launch_remap<R, 28>(a, s); break;
      default: launch_remap<R, 14>(a, s); break;
    }
  }
  if (ev && e == hipSuccess) e = hipEventRecord(ev[3], s);
  const hipError_t l = hipGetLastError();
  return l != hipSuccess ? l : e;
}

template <typename R>
hipError_t launch_totals(const Mesh &m, Ctl *ctl, const Work<R> &w, int cur, hipStream_t s) {
  if constexpr (std::is_same<R, double>::value) {
    if (m.mode == 1)
      hipLaunchKernelGGL(k_lag_totals_partial, dim3(TOT_BLOCKS), dim3(TPB), 0, s, m, w.s[cur],
                         (const double *)w.lg.m, w.partial);
    else
      hipLaunchKernelGGL(k_totals_partial<R>, dim3(TOT_BLOCKS), dim3(TPB), 0, s, m, w.s[cur], w.partial);
  } else {
    hipLaunchKernelGGL(k_totals_partial<R>, dim3(TOT_BLOCKS), dim3(TPB), 0, s, m, w.s[cur], w.partial);
  }
  hipLaunchKernelGGL(k_totals_final, dim3(1), dim3(TPB), 0, s, ctl, (const double *)w.partial);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_export(const Mesh &m, const Work<R> &w, int cur, int which, double *out, hipStream_t s) {
  const int64_t n = which >= 4 ? m.nnode : m.ncell;
  hipLaunchKernelGGL(k_export<R>, dim3(blocks(n)), dim3(TPB), 0, s, m, w.s[cur], which, out);
  return hipGetLastError();
}

#define SALE_INSTANTIATE(R)                                                                              \
  template size_t workspace_bytes<R>(const Mesh &);                                                      \
  template size_t state_bytes<R>(const Mesh &);                                                          \
  template size_t inter_bytes<R>(const Mesh &);                                                          \
  template void layout<R>(const Mesh &, void *, Ctl **, Work<R> *);                                      \
  template void layout_split<R>(const Mesh &, void *, void *, Ctl **, Work<R> *);                        \
  template hipError_t launch_init_sod<R>(const Mesh &, Ctl *, const Work<R> &, const double[5], double,  \
                                         long long, double, hipStream_t);                                \
  template hipError_t launch_init_sedov<R>(const Mesh &, Ctl *, const Work<R> &, const double[3], double, \
                                           long long, double, hipStream_t);                              \
  template hipError_t launch_init_noh<R>(const Mesh &, Ctl *, const Work<R> &, const double[3], int, double,    \
                                         long long, double, hipStream_t);                                       \
  template hipError_t launch_init_user<R>(const Mesh &, Ctl *, const Work<R> &, const double *const[5],  \
                                          bool, double, long long, double, hipStream_t);                 \
  template RunArgs<R> run_args<R>(const Mesh &, Ctl *, const Work<R> &, int, const Launch &);            \
  template hipError_t launch_step<R>(const Mesh &, Ctl *, const Work<R> &, int, const Launch &, hipStream_t, \
                                    const hipEvent_t *);                                                 \
  template hipError_t launch_totals<R>(const Mesh &, Ctl *, const Work<R> &, int, hipStream_t);          \
  template hipError_t launch_export<R>(const Mesh &, const Work<R> &, int, int, double *, hipStream_t);
SALE_INSTANTIATE(double)
SALE_INSTANTIATE(float)

}  // namespace sale
