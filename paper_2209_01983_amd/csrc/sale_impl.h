// sale_impl.h -- internal declarations of libsale (device control block,
// workspace layout, kernel launchers). Not part of the public ABI.
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
  double h;           // min(dx, dy, dz): length scale of q and the CFL rule
  double ax, ay, az;  // quarter face areas dy*dz/4, dz*dx/4, dx*dy/4
  double gamma, cfl, cq, cl;
  int64_t ncell, nnode;
};

// Device control block (one per run), at the start of the workspace.
// `done` is decided once per step by the step's first kernel and read by
// every later kernel of the step, so a step after t_end or after an error
// flag changes nothing.
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
  double pad[6];
};

// FP64 workspace: state plus the temporaries of the multi-pass step.
// Face arrays are stored per cell: the face at the cell's lower side along
// that axis (zero on the domain's lower boundary); a cell's upper face is its
// +axis neighbour's lower face, or a wall (zero) on the last layer.
struct Fields64 {
  double *rho, *e;          // state, cells
  double *u, *v, *w;        // state, nodes
  double *ps;               // P*: predicted pressure + q
  double *rhoL, *eL;        // Lagrangian density and energy
  double *dvx, *dvy, *dvz;  // swept volumes of the lower faces
  double *mux, *muy, *muz;  // donor mass fluxes of the lower faces
  double *ex, *ey, *ez;     // donor energy fluxes of the lower faces
  double *M, *rn, *epre;    // remapped mass, density, energy before the KE fix
  double *u1, *v1, *w1;     // Lagrangian end velocity u'
  double *dkm;              // kinetic-energy defect per unit new nodal mass
  double *scratch;          // one spare cell array (derived fields)
  double *partial;          // reduction partials (diagnostics)
  int64_t npartial;
};

size_t workspace_bytes_fp64(const Mesh &m, size_t *ctl_off);
void layout_fp64(const Mesh &m, void *ws, Ctl **ctl, Fields64 *f);

// Initial states (asynchronous on `s`).
hipError_t launch_init_sod(const Mesh &m, Ctl *ctl, const Fields64 &f, const double sod[5],
                           double t0, long long step0, double t_end, hipStream_t s);
hipError_t launch_init_sedov(const Mesh &m, Ctl *ctl, const Fields64 &f, const double sedov[3],
                             double t0, long long step0, double t_end, hipStream_t s);
// User arrays already copied into the state: zero wall-normal velocities,
// reset the control block and compute the first signal speed.
hipError_t launch_init_user(const Mesh &m, Ctl *ctl, const Fields64 &f, double t0,
                            long long step0, double t_end, hipStream_t s);

hipError_t launch_set_t_end(Ctl *ctl, double t_end, hipStream_t s);
hipError_t launch_step_fp64(const Mesh &m, Ctl *ctl, const Fields64 &f, hipStream_t s);
hipError_t launch_totals_fp64(const Mesh &m, Ctl *ctl, const Fields64 &f, hipStream_t s);
// p (which = 0) or q (which = 1) of the current state into `out` (cells).
hipError_t launch_derived_fp64(const Mesh &m, const Fields64 &f, int which, double *out,
                               hipStream_t s);

}  // namespace sale
