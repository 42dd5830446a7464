// sale_impl.h -- internal declarations of libsale (device control block,
// workspace layout, run descriptors, kernel launchers). Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace sale {

// Mesh geometry and scheme constants, passed by value to every kernel.
struct Mesh {
  int nx, ny, nz;
  double lo[3];       // lower corner of the box
  double dx, dy, dz;  // cell edge lengths
  double V0;          // cell volume dx*dy*dz
  double iV0;         // 1 / V0
  double h;           // min(dx, dy, dz): length scale of q and the CFL rule
  double ax, ay, az;  // quarter face areas dy*dz/4, dz*dx/4, dx*dy/4
  double gamma, cfl, cq, cl;
  // products of constants, formed once on the host (device code would form
  // them in vector registers and keep them live)
  double gm1, ggm1;          // gamma - 1, gamma (gamma - 1)
  double cq4h;               // 4 c_quad h
  double hyz, hzx, hxy;      // face areas dy dz, dz dx, dx dy
  double edx, edy, edz;      // eighth spacings dx/8, dy/8, dz/8 (swept volumes)
  int64_t ncell, nnode;
  int order;                 // remap order: 1 donor cell, 2 limited linear
  int mode;                  // 0 Eulerian (Lagrange + remap), 1 pure Lagrangian (mesh moves)
  double chg;                // hourglass viscosity coefficient (pure Lagrangian mode)
};

// Device control block (one per run). `done` is decided once per step by the
// step's first kernel and read by every later kernel of the step, so a step
// after t_end or after an error flag changes nothing. The two counters are
// used by the persistent multi-run kernel only.
struct Ctl {
  double t;           // time of the state after the step in flight
  double dt;          // dt of the step in flight
  double t_end;
  double dt_next;     // dt the next step will take (informational)
  unsigned long long amax_bits;  // max signal speed of the current state (bits of a double >= 0)
  long long step;     // steps completed (including the one in flight)
  unsigned int status;  // sticky SALE_FLAG_* bits
  unsigned int done;    // this step is a no-op
  double totals[2];   // mass, energy (written by the diagnostics kernels)
  unsigned int tiles_done;  // persistent kernel: finished tiles of the current phase
  unsigned int phase;       // persistent kernel: phase counter of the run
  long long step_target;    // persistent kernel: stop after this many steps
  long long clk_first;      // persistent kernel: device wall clock at the run's first advance
  long long clk_last;       // persistent kernel: device wall clock when its last step completed
  double pad;
};

// One copy of the state, logical layout (see include/sale.h). R is the
// storage type of the bulk quantities: double (SALE_FP64) or float
// (SALE_MIXED32).
template <typename R>
struct State {
  R *rho, *e;    // cells
  R *u, *v, *w;  // nodes
};

// Per-cell results of the Lagrangian phase handed from the first step kernel
// to the second: e^L and the swept volumes of the cell's three lower faces (x
// face at its lower x side, etc.; zero on the domain boundary). A cell's
// upper face is its +axis neighbour's lower face, or a wall; the remap forms
// V^L and rho^L from the six. Swept volumes are computed in FP64 in both
// precisions and handed over in the bulk type R, the type the remap's fluxes
// use them in. rho^L (second-order remap only, null otherwise) is formed by a
// pass of its own for the second-order passes, which read it with a halo.
template <typename R>
struct Geo {
  R *rl, *el;
  R *dvx, *dvy, *dvz;
};

// Workspace of one run: two states (ping-pong), the Lagrangian end velocity
// u' and the Lagrangian cell results, reduction partials, and one scratch
// array of max(cells, nodes) doubles (conversions, derived fields).
// Intermediates of the second-order remap (null for order 1): mass fluxes
// through each cell's three lower faces, the cells' new masses and pre-fix
// energies, and the nodes' kinetic-energy defects per unit new mass.
template <typename R>
struct Rem2 {
  R *mu[3];  // mass flux through each cell's lower face, per axis
  R *M, *epre;
  R *dk;
};

// Pure-Lagrangian mode (FP64 only; null otherwise): node positions of the two
// states, the constant cell masses, and the corner forces of the step in
// flight, F[(3 a + d) * corner_stride(ncell) + c] for corner a = (a&1, a>>1&1,
// a>>2&1) and component d of cell c.
struct Lag {
  double *x[2], *y[2], *z[2];
  double *m;
  double *F;
};
// Stride in doubles between the 24 corner-force arrays: the cell count
// rounded up to 256 bytes plus 33 blocks of 256 bytes, so that the arrays do
// not start at one offset modulo a large power of two (with a power-of-two
// cell count the 24 streams of a kernel would all meet in the same memory
// channels).
__host__ __device__ inline int64_t corner_stride(int64_t ncell) { return (ncell + 31) / 32 * 32 + 33 * 32; }

template <typename R>
struct Work {
  State<R> s[2];
  R *up, *vp, *wp;
  Geo<R> geo;
  double *partial;
  double *scratch;
  Rem2<R> r2;
  Lag lg;
};

// Pure-Lagrangian mode: positions and masses of the initial Cartesian mesh
// from state w.s[0] and the first signal (max over cells of a / h) into ctl;
// one step from buffer cur into 1 - cur (kernels in sale_lagrange.hip).
hipError_t launch_lag_init(const Mesh &m, Ctl *ctl, const Work<double> &w, hipStream_t s);
hipError_t launch_lag_step(const Mesh &m, Ctl *ctl, const Work<double> &w, int cur, hipStream_t s,
                           const hipEvent_t *ev);
// Node coordinate `axis` of state buffer `cur` as doubles into out: the
// moving mesh in the pure-Lagrangian mode, the fixed mesh otherwise.
template <typename R>
hipError_t launch_positions(const Mesh &m, const Work<R> &w, int cur, int axis, double *out, hipStream_t s);

// The second-order remap (multi-pass kernels in sale_remap2.hip): from the
// Lagrangian results in w.geo (rho^L included: the second-order step's
// Lagrange kernel forms it) / u' into w.s[1 - cur], then the next signal
// speed into ctl.
template <typename R>
hipError_t launch_remap2(const Mesh &m, Ctl *ctl, const Work<R> &w, int cur, hipStream_t s);

// Launch decomposition of a z-marching step kernel: tiles of 36 x CH columns
// (32 owned in x),
// the z extent split into segments so that the grid fills the chip.
struct Grid2 {
  int tx, ty, nseg, seglen;  // tiles per axis, z segments, planes per segment
  __host__ __device__ int blocks() const { return tx * ty * nseg; }
};

// Everything a step kernel needs about one run, for one step from state
// buffer `cur` into `nxt`.
template <typename R>
struct RunArgs {
  Mesh m;
  Ctl *ctl;
  State<R> cur, nxt;
  R *up, *vp, *wp;
  Geo<R> geo;
  Grid2 ga, gb;  // decompositions of the Lagrange and remap kernels
};

// Launch shape of the two z-marching kernels of a single run: tile rows
// (tiles are 36 x rows columns, one thread per column; rows 7, 14 or 28) and
// the number of blocks the z segmentation aims at.
struct Launch {
  int rows_a = 14;     // Lagrange + geometry kernel
  int rows_b = 14;     // remap kernel
  int target = 0;      // blocks per kernel the z split aims at (0: automatic)
};
bool launch_valid(const Launch &L);

// (width: the tile's columns in x, halo included)
Grid2 grid_lagrange(const Mesh &m, int target_blocks, int rows, int width);
Grid2 grid_remap(const Mesh &m, int target_blocks, int rows, int width);
constexpr int kStepThreads = 512;  // block size of the 16-row tiles (and of the pool kernel)

template <typename R>
size_t workspace_bytes(const Mesh &m);
// the state part (control block, two state buffers) and the intermediates
template <typename R>
size_t state_bytes(const Mesh &m);
template <typename R>
size_t inter_bytes(const Mesh &m);
template <typename R>
void layout(const Mesh &m, void *ws, Ctl **ctl, Work<R> *w);
template <typename R>
void layout_split(const Mesh &m, void *state, void *inter, Ctl **ctl, Work<R> *w);

// The library's device array for the intermediates of sale_init_static
// contexts (sale_noalloc.hip): its size, and its address on the current
// device (looked up once per device).
constexpr size_t kStaticScratchBytes = size_t(160) << 20;
hipError_t static_scratch(void **ptr);

// Initial states into w.s[0] (asynchronous on `s`).
template <typename R>
hipError_t launch_init_sod(const Mesh &m, Ctl *ctl, const Work<R> &w, const double sod[5], double t0,
                           long long step0, double t_end, hipStream_t s);
template <typename R>
hipError_t launch_init_sedov(const Mesh &m, Ctl *ctl, const Work<R> &w, const double sedov[3], double t0,
                             long long step0, double t_end, hipStream_t s);
// User arrays (double): copied through the scratch array into w.s[0], wall-
// normal velocities zeroed, control block reset, first signal speed computed.
template <typename R>
hipError_t launch_init_noh(const Mesh &m, Ctl *ctl, const Work<R> &w, const double noh[3], int dims, double t0,
                           long long step0, double t_end, hipStream_t s);
template <typename R>
hipError_t launch_init_user(const Mesh &m, Ctl *ctl, const Work<R> &w, const double *const src[5],
                            bool on_device, double t0, long long step0, double t_end, hipStream_t s);

hipError_t launch_set_t_end(Ctl *ctl, double t_end, hipStream_t s);
// One step from w.s[cur] into w.s[1 - cur].
// With `ev` (4 events), ev[0..3] are recorded before the step and after each
// of its three kernels (start, Lagrange+geometry, remap).
template <typename R>
hipError_t launch_step(const Mesh &m, Ctl *ctl, const Work<R> &w, int cur, const Launch &L, hipStream_t s,
                       const hipEvent_t *ev = nullptr);
template <typename R>
hipError_t launch_totals(const Mesh &m, Ctl *ctl, const Work<R> &w, int cur, hipStream_t s);
// Step arguments of one run (state w.s[cur] -> w.s[1 - cur]) for launch shape L.
template <typename R>
RunArgs<R> run_args(const Mesh &m, Ctl *ctl, const Work<R> &w, int cur, const Launch &L);
// Field `which` of state w.s[cur] as doubles into `out`: 0 rho, 1 e, 2 p, 3 q
// (cells), 4 u, 5 v, 6 w (nodes).
template <typename R>
hipError_t launch_export(const Mesh &m, const Work<R> &w, int cur, int which, double *out, hipStream_t s);

}  // namespace sale
